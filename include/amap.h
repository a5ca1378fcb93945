/*
 * amap.h -- C ABI of the fast weak-lensing aperture-mass library for AMD
 * Instinct MI355X (gfx950).
 *
 * The library implements the fast aperture-mass path of Leonard, Pires &
 * Starck, "Fast Calculation of the Weak Lensing Aperture Mass Statistic"
 * (arXiv:1204.4293): a pixelised shear map is turned into a convergence map
 * by Kaiser-Squires inversion in Fourier space (Sec. 1, Sec. 4.5), the
 * convergence map is decomposed by the starlet transform into J planes whose
 * detail planes are aperture-mass maps at radii 2^j pixels (Sec. 3), noise
 * maps come from randomising the shears many times and S = M_ap / sigma
 * (Sec. 1), and peaks are counted per scale on S (Sec. 2.2).  The brute-force
 * aperture mass of eq:shearmap is provided for comparison (Sec. 5.1).
 *
 * Conventions (all entry points):
 *   - A map is square n x n, n a power of two with 16 <= n <= 4096, stored
 *     row-major [y][x] with contiguous rows (x is the column index).  All
 *     boundaries are periodic.
 *   - J counts the planes produced *including* the smooth plane (Sec. 3:
 *     J = j_max + 1), 2 <= J and 2^J <= n (Sec. 5.1).  A plane stack is
 *     [J][n][n]: w_1 .. w_{J-1}, then c_{J-1}; w_j is the aperture-mass map
 *     at theta = 2^j pixels.  Smoothing step j uses the B3-spline taps
 *     (1,4,6,4,1)/16 at dilation 2^(j-1), row pass then column pass.
 *   - Data pointers are DEVICE pointers, owned by the caller, of the element
 *     type given by the dtype argument (float or double), 256-byte aligned.
 *     The library reads or writes them only inside the work it enqueues and
 *     keeps no reference after the call (plans: until amap_plan_destroy).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call validates its arguments on the host, enqueues its kernels on
 *     `stream` and returns without waiting.  Work issued through one context
 *     uses that context's workspace, so calls sharing a context must be
 *     ordered on one stream (use one context per concurrent stream).
 *   - Errors: a call returns a status; on failure nothing has been enqueued
 *     and amap_last_error() describes the problem.  Asynchronous device
 *     errors surface as AMAP_E_HIP from a later call or from amap_sync.
 *     No C++ exception crosses this interface.
 */
#ifndef AMAP_H
#define AMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMAP_OK = 0,
    AMAP_E_INVAL = 1,       /* invalid argument; nothing was enqueued        */
    AMAP_E_NOMEM = 2,       /* device memory for workspace unavailable       */
    AMAP_E_HIP = 3,         /* HIP runtime error (launch or asynchronous)    */
    AMAP_E_UNSUPPORTED = 4, /* valid request this build does not handle      */
    AMAP_E_BUSY = 5         /* server queue full; submit again later         */
} amap_status;

typedef enum { AMAP_F32 = 0, AMAP_F64 = 1 } amap_dtype;

/* Aperture-mass filters of Sec. 4: the starlet Q(eta) of Sec. 4.2, the
 * polynomial S98 filter of eq:sch (fparam = l) and the Gaussian filter of
 * eq:mexhat with A = 1 (fparam = b). */
typedef enum {
    AMAP_FILTER_STARLET = 0,
    AMAP_FILTER_S98 = 1,
    AMAP_FILTER_JBJ04 = 2
} amap_filter;

/* Edge rules for fields that are not periodic squares (the paper raises
 * survey-field edges at the end of Sec. 5 and fixes no rule): an index
 * outside [0, n) is taken modulo n (periodic), reflected about the first and
 * last samples with period 2(n-1), the edge samples not repeated (mirror),
 * or the sample is 0 (zero). */
typedef enum {
    AMAP_BC_PERIODIC = 0,
    AMAP_BC_MIRROR = 1,
    AMAP_BC_ZERO = 2
} amap_boundary;

typedef struct amap_ctx*  amap_ctx_t;
typedef struct amap_plan* amap_plan_t;
typedef struct amap_server* amap_server_t;

/* Create a context on HIP device `hip_device`.  The context owns the
 * twiddle tables and a growable device workspace.  *out is set on success. */
amap_status amap_create(int hip_device, amap_ctx_t* out);

/* Destroy a context after waiting for its device; NULL is accepted. */
amap_status amap_destroy(amap_ctx_t ctx);

/* Text of the last error of the calling thread ("" if none).  Valid until
 * the next amap_* call on that thread. */
const char* amap_last_error(void);

/* Wait for `stream` and report any asynchronous device error. */
amap_status amap_sync(amap_ctx_t ctx, void* stream);

/* Bytes of workspace the context currently holds on the device. */
size_t amap_workspace_bytes(amap_ctx_t ctx);

/* Tile autotuning (on by default).  The first starlet transform of each
 * shape (element type, n, J, signal or noise statistics, batch) on a stream
 * that is not being captured times the candidate LDS tiles of every stage
 * start and scale count on the call's own buffers (for noise statistics
 * also stages on sub-grid images and final sub-grid stages) and keeps, per
 * context, the schedule of least total time (dynamic programming over the
 * stage starts); later calls of that shape reuse it.  Batch plans tune at
 * creation with one direct run of the plan.  Results do not depend on the
 * schedule except, for noise statistics, in the rounding of how per-group
 * partial statistics are merged.  enable = 0 uses the analytic planner
 * (fewest stages, least halo overhead) and keeps existing tuned schedules
 * unused until it is enabled again; enable = 2 uses the analytic planner
 * for noise statistics too, but ends them with a final stage on whole
 * sub-grids (two realisations per pass) wherever one applies: a fixed
 * schedule that always exercises that stage.  Other values: AMAP_E_INVAL. */
amap_status amap_set_autotune(amap_ctx_t ctx, int enable);

/* Writes the context's tuned schedules as JSON into buf (len bytes including
 * the NUL): [{"mode": 1 (tuned) | 2 (analytic with sub-grid final stage, see
 * amap_set_autotune), "elem": bytes per value, "logn", "J", "noise": 0|1, "batch",
 * "stages": [[j0, ns, tile width, tile sub-rows, realisations per LDS
 * pass, kind], ...]}, ...].  Every scale from j0 on couples only pixels
 * congruent mod d = 2^(j0-1) (the a-trous dilations, Sec. 2.3), so the d^2
 * sub-grids of such pixels are independent periodic images of side n / d.
 * kind 0: an LDS tile stage; kind 1 (noise statistics, the last stage): a
 * final stage on whole sub-grids, one per workgroup (width and sub-rows are
 * the sub-grid side); kind 2 (noise statistics): a tile stage on the
 * sub-grids of d taken as images, with the tile of an (n/d) x (n/d) map's
 * first stage; it follows a kind-0 or kind-2 stage and is the last stage or
 * followed by a kind-2 or kind-1 stage (each such stage lays out the
 * sub-grids of the next inside its own images).  An empty stage list means
 * the analytic planner is used for that shape.
 * AMAP_E_INVAL if it does not fit. */
amap_status amap_plans_read(amap_ctx_t ctx, char* buf, size_t len);

/* Loads schedules in amap_plans_read's format (NUL-terminated JSON) into the
 * context, replacing any it holds for the same shapes; later transforms of
 * those shapes use them instead of tuning (mode 1) or of the mode-2
 * analytic schedule.  Lets a caller keep tuned schedules across processes
 * and run a fixed schedule (for instance under a profiler, whose timing
 * would steer the tuner).  Every schedule is checked against the planner's
 * tiles and the stage rules first; AMAP_E_INVAL (nothing loaded) if one is
 * malformed or invalid. */
amap_status amap_plans_load(amap_ctx_t ctx, const char* json);

/* Per-kernel timing (diagnostics): while enabled, every kernel the context
 * launches is bracketed by two HIP events recorded on the launch's stream.
 * Work captured into a batch plan's graph is not timed. */
amap_status amap_timing_enable(amap_ctx_t ctx, int enable);

/* Restricts the timing to launches of one kernel name (as reported by
 * amap_timing_read); NULL or "" times every launch again.  Launches of
 * other kernels then run without events around them.  AMAP_E_INVAL if
 * timing is not enabled. */
amap_status amap_timing_select(amap_ctx_t ctx, const char* kernel);

/* Waits for the timed work and writes a JSON object
 * {"kernel": [launches, total_ms], ...} into buf (len bytes, including the
 * terminating NUL; AMAP_E_INVAL if it does not fit).  reset != 0 clears the
 * totals afterwards. */
amap_status amap_timing_read(amap_ctx_t ctx, char* buf, size_t len, int reset);

/*
 * Kaiser-Squires inversion (Sec. 1: the shear map is converted into a
 * convergence map in Fourier space; Sec. 4.5).
 *   kappa = F^-1[ conj(D) F(g1 + i g2) ],
 *   D(k) = [(k1^2 - k2^2) + 2 i nu k1 k2] / |k|^2, D(0) = 0,
 * with k1 along x, nu = 0 on the Nyquist row and column, 1 elsewhere.
 * Inputs g1, g2: n*n each.  Outputs kappa_e = Re kappa (n*n) and, if not
 * NULL, kappa_b = Im kappa (n*n).  Outputs may not alias inputs.
 */
amap_status amap_ks_invert(amap_ctx_t ctx, amap_dtype dt, int n,
                           const void* g1, const void* g2,
                           void* kappa_e, void* kappa_b, void* stream);

/*
 * amap_ks_invert without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels, arguments, layout and results as
 * amap_ks_invert, but the complex spectrum lives in a static scratch array
 * of 64 MiB that each GPU holds from the first amap_create on it until the
 * process ends, instead of the context's workspace.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine).  Limit:
 * 2 n^2 elements of scratch, i.e. n <= 2048 for float32 and float64;
 * larger n returns AMAP_E_INVAL.  Every such call on one GPU shares that
 * GPU's array (all contexts), which keeps the last call's contents: calls
 * that overlap in time on one GPU (on different streams or host threads)
 * race and must be ordered by the caller.
 */
amap_status amap_ks_invert_noalloc(amap_ctx_t ctx, amap_dtype dt, int n,
                                   const void* g1, const void* g2,
                                   void* kappa_e, void* kappa_b, void* stream);

/*
 * Starlet decomposition (Sec. 3; eq:splinewl with the B3 spline of
 * Sec. 4.2): planes[J][n][n] = w_1 .. w_{J-1}, c_{J-1}, with c_0 = kappa,
 * c_j = column(row(c_{j-1})) at dilation 2^(j-1), w_j = c_{j-1} - c_j.
 * kappa: n*n; planes: J*n*n; they may not overlap.
 */
amap_status amap_starlet_forward(amap_ctx_t ctx, amap_dtype dt, int n, int J,
                                 const void* kappa, void* planes, void* stream);

/*
 * Starlet decomposition of an ny x nx field of any sides in [2, 16384]
 * (Sec. 3 cascade with the B3 taps of Sec. 4.2, as amap_starlet_forward)
 * under an edge rule `boundary` (amap_boundary), applied to c_{j-1} on each
 * axis at every smoothing step; 2 <= J <= 16.  image: ny*nx row-major;
 * planes: J*ny*nx, w_1 .. w_{J-1}, c_{J-1}; they may not overlap.  The
 * decomposition is exact under every rule (sum of the planes = image); the
 * detail planes have zero mean only under the periodic rule.  Uses ny*nx
 * elements of the context's workspace.
 */
amap_status amap_starlet_forward_bc(amap_ctx_t ctx, amap_dtype dt, int ny, int nx, int J,
                                    int boundary, const void* image, void* planes,
                                    void* stream);

/*
 * Kaiser-Squires inversion (as amap_ks_invert) of an ny x nx shear field that
 * is zero outside its rectangle: the field is placed at the origin of a
 * P x P periodic grid (P a power of two in [16, 4096], P >= ny, nx), inverted
 * there, and the ny x nx rectangle of kappa_E (and of kappa_B, if not NULL)
 * is written to kappa_e / kappa_b (ny*nx each, row-major).  P = n for an
 * n x n field is amap_ks_invert itself; P = 2 max(ny, nx) keeps the periodic
 * images of the field from overlapping it.  Outputs may not alias inputs.
 * Uses 6 P^2 elements of the context's workspace.
 */
amap_status amap_ks_invert_padded(amap_ctx_t ctx, amap_dtype dt, int ny, int nx, int P,
                                  const void* g1, const void* g2, void* kappa_e,
                                  void* kappa_b, void* stream);

/*
 * Noise maps of an ny x nx field with edges (Sec. 1; Sec. 5.1, as
 * amap_noise_maps): realisation r = 0 .. n_real-1 rotates every pixel's
 * shear by 2 pi u, u the Philox4x64-10 uniform of flat pixel index
 * y*nx + x (amap_phase_uniforms with n*n replaced by ny*nx); the rotated
 * field goes through amap_ks_invert_padded (grid P) and
 * amap_starlet_forward_bc (rule `boundary`).  sigma_j is the per-pixel
 * unbiased sample standard deviation (running mean and squared deviations
 * in double, Welford's update).  If snr is not NULL, planes_signal (J*ny*nx,
 * the signal's planes from the same two calls) must be given and
 * snr_j = w_j / sigma_j (0 where sigma_j = 0).  sigma, snr: (J-1)*ny*nx.
 * Sides >= 2 and <= P; n_real >= 2.  Realisations run in batches sized to
 * about 1 GiB of the context's workspace (at least one).
 */
amap_status amap_noise_maps_bc(amap_ctx_t ctx, amap_dtype dt, int ny, int nx, int P, int J,
                               int boundary, const void* g1, const void* g2, int n_real,
                               uint64_t seed, const void* planes_signal, void* sigma, void* snr,
                               void* stream);

/*
 * Peak counts of nplanes ny x nx planes with edges (as amap_count_peaks:
 * value > threshold and > each of its 8 neighbours, strict, in double, NaN
 * never a peak), each neighbour's row and column taken through the edge
 * rule `boundary` (under AMAP_BC_ZERO a neighbour outside the field is 0).
 * counts_dev: device array of nplanes long long, overwritten.
 */
amap_status amap_count_peaks_bc(amap_ctx_t ctx, amap_dtype dt, int ny, int nx, int nplanes,
                                int boundary, const void* planes, double threshold,
                                long long* counts_dev, void* stream);

/*
 * Masked fields (missing data inside the field: stars and bad pixels cut out
 * of the image, end of Sec. 5, where the paper notes that plain
 * reconstruction does not recover the lost information).  mask: ny*nx bytes,
 * row-major, non-zero where the pixel is observed and 0 where it is missing,
 * 256-byte aligned device memory.
 *
 * amap_mask_shear: g1_out = g1 and g2_out = g2 where observed, 0 where
 * missing (ny*nx each).  An output may be its own input (in place);
 * otherwise outputs overlap nothing.  The masked field then goes through
 * amap_ks_invert_padded / amap_noise_maps_bc (or the periodic calls for a
 * power-of-two square): a missing pixel carries no shear in the signal or in
 * any noise realisation, since a rotation keeps a zero shear zero.
 *
 * amap_count_peaks_masked: peaks as amap_count_peaks_bc, counted only where
 * the pixel and each of its 8 neighbours that the edge rule keeps inside the
 * field are observed (a maximum that touches missing data is not counted;
 * under AMAP_BC_ZERO a neighbour outside the field does not veto).  mask is
 * the same for every plane.  counts_dev: nplanes long long, overwritten.
 */
amap_status amap_mask_shear(amap_ctx_t ctx, amap_dtype dt, int ny, int nx,
                            const unsigned char* mask, const void* g1, const void* g2,
                            void* g1_out, void* g2_out, void* stream);
amap_status amap_count_peaks_masked(amap_ctx_t ctx, amap_dtype dt, int ny, int nx, int nplanes,
                                    int boundary, const void* planes, const unsigned char* mask,
                                    double threshold, long long* counts_dev, void* stream);

/* Exact inverse of the decomposition (Sec. 3): kappa_out = c_{J-1} + sum w_j.
 * planes: J*n*n; kappa_out: n*n (may not overlap planes). */
amap_status amap_starlet_reconstruct(amap_ctx_t ctx, amap_dtype dt, int n, int J,
                                     const void* planes, void* kappa_out, void* stream);

/*
 * Brute-force aperture mass from the tangential shear (eq:shearmap; cost
 * O(n^2 cut^2), Sec. 5.1):
 *   M(x) = sum_{0 < |d|^2 <= cut^2} Q_theta(|d|) gamma_t(x + d; x),
 *   gamma_t = -[g1 (dx^2 - dy^2) + g2 2 dx dy] / |d|^2,
 * indices periodic, pixel area 1.  Q_theta(r) = Q(r/theta)/theta^2 for the
 * starlet; S98 and JBJ04 as printed (they carry their own 1/theta^2).
 * theta_px > 0.  cut_px <= 0 selects the natural support: 2 theta
 * (starlet), theta (S98), 5 theta (JBJ04).  The cut radius must satisfy
 * 2*floor(cut) + 1 <= n and cut <= 256.  The inclusion test |d|^2 <= cut^2
 * is made in double precision.  map_out: n*n.
 */
amap_status amap_map_direct(amap_ctx_t ctx, amap_dtype dt, int n,
                            const void* g1, const void* g2, double theta_px,
                            amap_filter filter, double fparam, double cut_px,
                            void* map_out, void* stream);

/*
 * Noise maps from randomised shears (Sec. 1; Sec. 5.1).  For realisation
 * r = 0 .. n_real-1 every pixel's shear is rotated by beta = 2 pi u,
 * gamma' = gamma exp(i beta), with u the Philox4x64-10 uniform of
 * amap_phase_uniforms; gamma' goes through the same KS inversion and
 * starlet transform as the signal.  Per pixel and scale, the unbiased
 * sample standard deviation over the realisations,
 *   sigma_j = sqrt( sum_r (w_r - mean_r w)^2 / (R - 1) ),
 * kept as a running mean and sum of squared deviations (Welford's update
 * within a batch of realisations, merged across batches in double
 * precision).  If snr is not NULL, planes_signal
 * (J*n*n, the signal's planes) must be given and snr_j = w_j / sigma_j
 * (0 where sigma_j = 0).  sigma, snr: (J-1)*n*n.  n_real >= 2.
 */
amap_status amap_noise_maps(amap_ctx_t ctx, amap_dtype dt, int n, int J,
                            const void* g1, const void* g2, int n_real, uint64_t seed,
                            const void* planes_signal, void* sigma, void* snr,
                            void* stream);

/*
 * Peak counts (Sec. 2.2; Sec. 4.3): for each of the `nplanes` n x n planes
 * of `snr`, counts_dev[p] = number of pixels with value > threshold and
 * value > each of its 8 periodic neighbours (strict; comparisons in double
 * on the plane's exact values; NaN is never a peak).  counts_dev: device
 * array of nplanes long long, overwritten.
 */
amap_status amap_count_peaks(amap_ctx_t ctx, amap_dtype dt, int n, int nplanes,
                             const void* snr, double threshold,
                             long long* counts_dev, void* stream);

/*
 * The 32-bit Philox values behind the noise phases (Sec. 1 randomisation):
 * Philox4x64-10 (Salmon et al. 2011) with key (seed, 0) and block counter
 * (b, r, 0, 0); block b gives pixels 8b .. 8b+7 (pixel = y*n + x), each
 * 64-bit word split low half then high half.  The phase uniform is
 * (v >> 8) * 2^-24.  out_u32: device array of n*n uint32.
 */
amap_status amap_phase_uniforms(amap_ctx_t ctx, int n, uint64_t seed, uint64_t r,
                                uint32_t* out_u32, void* stream);

/*
 * The whole path for one map: KS inversion, starlet planes, noise sigma from
 * n_real randomised realisations, S/N and peak counts above `threshold`.
 * kappa_e (n*n) and kappa_b (n*n) may be NULL; planes (J*n*n), sigma and snr
 * ((J-1)*n*n) and peaks (J-1 long long, device) are required.
 */
amap_status amap_run_path(amap_ctx_t ctx, amap_dtype dt, int n, int J,
                          const void* g1, const void* g2, int n_real, uint64_t seed,
                          double threshold, void* kappa_e, void* kappa_b,
                          void* planes, void* sigma, void* snr,
                          long long* peaks, void* stream);

/* ---- statistics of the planes ---- */

/*
 * Central moments of each of `nplanes` n x n planes (Sec. 2.2: the variance
 * of the aperture mass, eq:varmap, its skewness and its kurtosis are the
 * statistics drawn from M_ap maps; plane w_j is the M_ap map at theta = 2^j).
 * out (device, 8-byte aligned, 4*nplanes doubles) receives, per plane p,
 * out[4p] = mean and out[4p+k-1] = m_k = (1/n^2) sum (x - mean)^k for
 * k = 2, 3, 4: the variance is m2, the skewness m3 / m2^1.5, the excess
 * kurtosis m4 / m2^2 - 3.  Two passes over the planes (mean, then the
 * central sums), accumulated in double with a fixed reduction order, so
 * results are reproducible.  Uses the context workspace.
 */
amap_status amap_plane_moments(amap_ctx_t ctx, amap_dtype dt, int n, int nplanes,
                               const void* planes, double* out, void* stream);

/*
 * Histogram of peak heights on each plane (Sec. 2.2: peak counts of M_ap
 * maps; richer peak statistics than amap_count_peaks).  A pixel counts when
 * sign*value exceeds sign*value of all 8 periodic neighbours, strictly
 * (sign = +1: peaks; sign = -1: troughs, i.e. peaks of the negated plane);
 * its height h = sign*value goes to bin floor((h - lo) / ((hi - lo) / nbins)),
 * computed in double, when that bin is in [0, nbins).  NaN is never a peak.
 * hist: device, 8-byte aligned, nplanes*nbins long long, overwritten.
 * 1 <= nbins <= 16384; lo < hi finite.  Counts above thresholds t_k follow
 * by summing bins.
 */
amap_status amap_peak_histogram(amap_ctx_t ctx, amap_dtype dt, int n, int nplanes,
                                const void* planes, int sign, double lo, double hi, int nbins,
                                long long* hist, void* stream);

/* ---- batched maps: one launch sequence over many maps of uneven sizes ---- */

/* One map of a batch.  n_real == 0 runs KS + starlet only (sigma, snr,
 * peaks ignored); n_real >= 2 runs the whole path as amap_run_path. */
typedef struct {
    int n, J, n_real;
    uint64_t seed;
    double threshold;
    const void *g1, *g2;
    void *kappa_e;      /* n*n or NULL                     */
    void *planes;       /* J*n*n, required                 */
    void *sigma, *snr;  /* (J-1)*n*n when n_real >= 2       */
    long long* peaks;   /* J-1 device counts when n_real>=2 */
} amap_job;

/* Validate `jobs` and build a plan that runs all of them.  Jobs without
 * noise (n_real == 0) of one (n, J) are grouped: each group (in chunks of at
 * most 2 GiB of workspace) runs as one launch per kernel over all its maps,
 * which the kernels address through device tables of per-map pointers built
 * here.  Jobs with noise (and shapes without grouped kernels) run alone, on
 * up to four lanes with a workspace region each (as many as fit 16 GiB of
 * workspace; each job to the lane with the least work so far): in the
 * captured graph of a non-null stream the lanes are branches forked from
 * and joined back into that stream, so their jobs overlap on the device;
 * on the null stream the lanes run one after another.  Results do not
 * depend on the lane.  The plan owns its workspace, tables, lane streams
 * and a captured HIP graph per stream; it keeps the job pointers until
 * destroyed, and the caller keeps the buffers alive and unshared between
 * jobs. */
amap_status amap_batch_plan(amap_ctx_t ctx, amap_dtype dt, const amap_job* jobs,
                            int njobs, amap_plan_t* out);

/* Run every job of the plan on `stream` (one graph launch after the first
 * call on that stream).  On the null stream the kernels are launched
 * directly, without a graph (and are timed when timing is enabled). */
amap_status amap_batch_run(amap_plan_t plan, void* stream);

/* Destroy a plan after waiting for its work; NULL is accepted. */
amap_status amap_plan_destroy(amap_plan_t plan);

/* Device bytes a job needs besides its own inputs and outputs (the unit an
 * admission policy budgets against). */
size_t amap_job_footprint_bytes(amap_dtype dt, int n, int J, int n_real);

/* Realisations the noise statistics of an n x n map process per launch
 * sequence (the batch its kernels and workspace are sized for): about
 * 2^27 pixels of realisations, at least 1 and at most n_real.  0 if n is not
 * a supported side or n_real < 2.  A context's amap_set_noise_batch cap
 * lowers the batch its calls use. */
int amap_noise_batch(int n, int n_real);

/* Caps the noise realisations the context's calls process per launch
 * sequence at max_batch (0 restores the default of amap_noise_batch).
 * Results equal those of the default batch up to the rounding of how the
 * per-batch statistics are merged (Chan's pairwise update, in double
 * precision); the workspace stays sized for the default batch.  Smaller
 * batches cost more merges; the cap exists so that the merge across
 * batches can be exercised on small maps.  AMAP_E_INVAL if max_batch < 0. */
amap_status amap_set_noise_batch(amap_ctx_t ctx, int max_batch);

/* ---- serving: continuous batching of independent jobs ---- */

/* A request loop on one context.  The server allocates one arena of
 * `mem_budget` bytes of device memory at creation.  Submitted jobs wait in a
 * FIFO; the oldest is admitted when one of `max_inflight` slots is free and
 * a free range of the arena holds its footprint (amap_job_footprint_bytes,
 * first fit); nothing is allocated while serving.  Each slot owns a HIP
 * stream (default priority), so admitted jobs run concurrently, and a
 * finishing job returns its slot and range without synchronising the
 * device.  Admission happens inside submit, poll
 * and wait, so callers that keep submitting and polling get continuous
 * batching.  A job's results are the same alone or in a mix: the kernels of
 * a job read only its own inputs and workspace.  The job's buffers must stay
 * valid until poll reports it done.  Calls on one server are not
 * thread-safe. */
amap_status amap_server_create(amap_ctx_t ctx, amap_dtype dt, size_t mem_budget,
                               int max_inflight, int max_queued, amap_server_t* out);

/* Validate and enqueue `job` (copied); `*ticket` identifies it.  An event
 * is recorded on `stream` (a hipStream_t as void*, NULL = the null stream)
 * at submission and the job's kernels wait for it, so the job runs after
 * everything enqueued on `stream` before the call (for instance the work
 * that produced its inputs or initialised its outputs), whatever slot it is
 * admitted to.  AMAP_E_NOMEM if its footprint alone exceeds the budget
 * (never admissible); AMAP_E_BUSY if max_queued jobs already wait.  A job
 * whose starlet shape has no tile schedule in the context yet (with
 * autotuning on) is tuned when it is admitted, which blocks the admitting
 * call until the job's submit point has been reached on the device and the
 * timing runs are done; amap_plans_load beforehand avoids that. */
amap_status amap_server_submit(amap_server_t srv, const amap_job* job, void* stream,
                               long long* ticket);

/* Admit what fits, then report whether `ticket` has finished (*done = 1;
 * its outputs are then complete and visible to later work on any stream).
 * AMAP_E_INVAL for an unknown ticket. */
amap_status amap_server_poll(amap_server_t srv, long long ticket, int* done);

/* Admit what fits, then write up to `cap` tickets that finished since the
 * last call into `out` (oldest first) and their number into *count.  Lets a
 * loop with many jobs outstanding poll once per iteration. */
amap_status amap_server_completed(amap_server_t srv, long long* out, int cap, int* count);

/* Block until `ticket` has finished. */
amap_status amap_server_wait(amap_server_t srv, long long ticket);

/* Jobs waiting, jobs on the device, and the admitted footprint in bytes. */
amap_status amap_server_stats(amap_server_t srv, int* queued, int* inflight,
                              size_t* mem_in_use);

/* Finish all submitted work and release the server; NULL is accepted. */
amap_status amap_server_destroy(amap_server_t srv);

#ifdef __cplusplus
}
#endif

#endif /* AMAP_H */

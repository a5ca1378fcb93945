// Host-side launchers of the library's kernels (internal to the library).
// Each launcher enqueues on `stream` and returns hipGetLastError().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amap {

template <typename T> struct cpx;

// Optional per-kernel timing.  When a KernelTimer is installed for the
// calling thread, every launch is bracketed by HIP events recorded on the
// launch's own stream.
struct KernelTimer {
    virtual ~KernelTimer() {}
    virtual void begin(const char* name, hipStream_t s) = 0;
    virtual void end(hipStream_t s) = 0;
};
KernelTimer*& current_timer();

#define AMAP_LAUNCH(name, stream, ...)                         \
    do {                                                       \
        ::amap::KernelTimer* t_ = ::amap::current_timer();     \
        if (t_) t_->begin(name, stream);                       \
        __VA_ARGS__;                                           \
        if (t_) t_->end(stream);                               \
    } while (0)

// Kaiser-Squires inversion of `batch` maps of side 2^logn.
//   g1/g2:   map b at g + b*g_stride (g_stride = 0: one map, many realisations)
//   C:       complex workspace, batch*n*n
//   kE/kB:   outputs at + b*out_stride; kB may be null
//   rotate:  rotate pixel shears by the Philox phases of realisation r0 + b
template <typename T>
struct KsArgs {
    int logn;
    int batch;
    const T* g1;
    const T* g2;
    long long g_stride;
    cpx<T>* C;
    T* kE;
    T* kB;
    long long out_stride;
    bool rotate;
    uint64_t seed;
    uint64_t r0;
    const cpx<T>* tw;  // exp(-2 pi i k / 4096), k < 4096
    hipStream_t stream;
    // grouped maps: device tables of per-map element offsets from g1, g2, kE
    // (null: b * stride).  Offsets from a kernel-argument pointer keep the
    // accesses in the global address space, so they stay vectorised.
    const long long* g1_off = nullptr;
    const long long* g2_off = nullptr;
    const long long* kE_off = nullptr;
    // kappa_B not wanted (kB ignored): where supported, maps 2p and 2p+1
    // share one inverse transform (their Hermitian parts packed as
    // H_2p + i H_2p+1); C is overwritten either way.  Needs kE_off == null.
    bool pair_e = false;
};
template <typename T> hipError_t launch_ks(const KsArgs<T>& a);

// Starlet decomposition of `batch` maps (kappa at + b*in_stride).
//   WRITE (S1 == null): planes at + b*planes_stride (J planes of n*n)
//   ACC   (M != null):  noise realisations; M/M2 [J-1][n*n] double running
//                       mean and sum of squared deviations of w_j over the
//                       `done` realisations merged so far; planes unused
// Scratch (each batch*n*n): cbuf0 (always), cbuf1 (ACC), tmp; wbuf (ACC):
// 3*batch*n*n, the detail planes of one stage.
// A starlet stage schedule: stage k covers scales st[k].j0 .. j0+ns-1 with
// an LDS tile of tw pixels by th sub-rows, rb realisations per LDS pass
// (noise stages; 1 otherwise).  kind (noise stages only):
//   kStageSubgrid: a final stage on whole sub-grids of d0 = 2^(j0-1)
//     (tw = th = n / d0), whose input and running statistics are in
//     sub-grid order;
//   kStageImages: a tile stage on the sub-grids of d0 = 2^(j0-1) taken as
//     periodic images of side n / d0 (its scales start at dilation 1 there;
//     tw, th a tile of such an image), whose input and running statistics
//     are in that sub-grid order; it follows a plain tile stage or another
//     such stage, and is the last stage or followed by another such stage
//     or the final sub-grid stage, whose sub-grids it lays out image by
//     image (nested sub-grid orders).
// nstages == 0: use the analytic planner.
enum { kStageTile = 0, kStageSubgrid = 1, kStageImages = 2 };
struct StagePlan {
    int nstages = 0;
    struct Stage { int j0, ns, tw, th, rb, kind; } st[16];
    // a one-stage noise plan (timed by the tuner) writes its coarse output
    // in sub-grid order for d = 2^cout_logd, as before a sub-grid stage
    int cout_logd = 0;
};

// Where a noise schedule leaves each scale's running statistics: from the
// first scale j0[k] of its k-th stage on sub-grids (images or whole
// sub-grids, in order) they are in the sub-grid order of d = 2^(j0[k]-1),
// nested inside each sub-grid of the stage before (stat_index).
struct StatLayout {
    int count = 0;
    int j0[16];  // as many as a schedule has stages
};
inline StatLayout stat_layout(const StagePlan* p) {
    StatLayout l;
    for (int k = 0; p && k < p->nstages && l.count < 16; ++k)
        if (p->st[k].kind != kStageTile) l.j0[l.count++] = p->st[k].j0;
    return l;
}

template <typename T>
struct StarletArgs {
    int logn, J, batch, done;
    const T* kappa;
    long long in_stride;
    T* planes;
    long long planes_stride;
    T* cbuf0;
    T* cbuf1;
    T* tmp;
    T* wbuf;
    double* M;
    double* M2;
    void* part;         // ACC: per-group partial statistics (starlet_partials_bytes)
    hipStream_t stream;
    // grouped maps (write mode only): map m reads kappa + kappa_off[m] and
    // writes its J planes at planes + planes_off[m] (element offsets); needs
    // cbuf0 and cbuf1 and a tiled plan
    const long long* kappa_off = nullptr;
    const long long* planes_off = nullptr;
    const StagePlan* plan = nullptr;  // tuned schedule, or null for the analytic one
};
// Bytes of per-group partial statistics a noise batch may need.
size_t starlet_partials_bytes(int logn, int batch);
template <typename T> hipError_t launch_starlet(const StarletArgs<T>& a);
// True when every stage of an n x n, J-plane transform has an LDS tile
// (grouped maps need it).
template <typename T> bool starlet_all_tiled(int n, int J);
// The analytic noise schedule ending in a sub-grid final stage, if one applies.
template <typename T> bool analytic_subgrid_plan(int n, int J, StagePlan* out);
// Whether a schedule is one launch_starlet accepts for this shape.
template <typename T> bool plan_valid(int n, int J, bool noise, const StagePlan& plan);
template <typename T>
hipError_t launch_peak_hist(int logn, int nplanes, const T* planes, int sign, double lo,
                            double width, int nbins, long long* hist, hipStream_t s);
// Blocks per plane of the moment reductions (their partials: 3 x nplanes x this doubles).
int moment_blocks(int logn);
template <typename T>
hipError_t launch_plane_moments(int logn, int nplanes, const T* planes, double* part, double* out4,
                                hipStream_t s);
// Times candidate tiles of every stage start and scale count on a's buffers
// (reps launches each, on a.stream, synchronously) and picks the schedule of
// least total time by dynamic programming over the stage starts.  Writes
// garbage into a's outputs and, for noise statistics, into M and M2.
template <typename T> hipError_t tune_starlet(const StarletArgs<T>& a, int reps, StagePlan* out);
template <typename T>
hipError_t launch_reconstruct(int logn, int J, const T* planes, T* out, hipStream_t s);

// Noise statistics.
// sigma = sqrt(M2/(R-1)); snr = w/sigma (0 where sigma = 0) if snr
template <typename T>
hipError_t launch_noise_finalize(int logn, int J, int R, const double* M2,
                                 const T* planes_signal, T* sigma, T* snr, hipStream_t s,
                                 const StatLayout& layout = StatLayout());
hipError_t launch_zero_f64(double* p, long long count, hipStream_t s);
hipError_t launch_zero_i64(long long* p, long long count, hipStream_t s);

template <typename T>
hipError_t launch_count_peaks(int logn, int nplanes, const T* snr, double thr,
                              long long* counts, hipStream_t s);

hipError_t launch_phase_u32(int logn, uint64_t seed, uint64_t r, uint32_t* out, hipStream_t s);

// Direct aperture mass: taps for offsets dy in [-R, R] (row dy + R), the
// dx range [-half[dy+R], half[dy+R]] (half < 0: empty row), weights wc
// (Q cos 2phi) and ws (Q sin 2phi) dense [(2R+1)][(2R+1)] in T.
// gtab (may be null): the weights regrouped for the LDS row kernel (maps
// from 512 px wide): row dy + R holds, per group of four dx from
// dx = -R4 (R4 = R rounded up to a multiple of 4), four Q cos 2phi then four
// Q sin 2phi, R4 / 2 + 1 groups, zero outside the disc;
// map_direct_uses_groups tells whether the row kernel runs (and needs it).
template <typename T>
hipError_t launch_map_direct(int logn, const T* g1, const T* g2, int R, const int* half,
                             const T* wc, const T* ws, const T* gtab, T* out, hipStream_t s);
bool map_direct_uses_groups(int logn, int R, size_t elem);

// Starlet of `maps` ny x nx fields (any sizes >= 2) under a boundary rule
// (0 periodic, 1 mirror: whole-sample symmetric, 2 zero outside): J planes
// w_1 .. w_{J-1}, c_{J-1}, each ny*nx; map m's image at image + m
// image_stride, its planes at planes + m planes_stride; `tmp` holds
// maps*ny*nx.
template <typename T>
hipError_t launch_starlet_bc(int ny, int nx, int J, int mode, const T* image, T* planes, T* tmp,
                             int maps, long long image_stride, long long planes_stride, hipStream_t s);

// Zero extension of an ny x nx pair of fields into P x P arrays, and the
// ny x nx rectangles of `maps` P x P arrays (in_stride apart) read back
// (out_stride apart; kB_p/kB may be null).
template <typename T>
hipError_t launch_pad2(const T* g1, const T* g2, int ny, int nx, int P, T* p1, T* p2, hipStream_t s);
template <typename T>
hipError_t launch_crop2(const T* kE_p, const T* kB_p, int P, int ny, int nx, T* kE, T* kB, int maps,
                        long long in_stride, long long out_stride, hipStream_t s);

// Noise realisations of a bounded field: the ny x nx shears rotated by the
// Philox phases of realisations r0 .. r0+nb-1 (flat pixel index y*nx + x)
// and written into the field's rectangle of each realisation's P x P
// arrays (p_stride apart; their rest is left as it is: cleared once by
// launch_zero2); Welford's update of the running mean M and squared
// deviations M2 (double, `count` elements) with the values of realisations
// r0 .. r0+nb-1 in order, w_stride apart (realisation 0 writes them unread);
// sigma = sqrt(M2/(R-1)) and, if snr is not null, snr = w_signal / sigma (0
// where sigma = 0).
template <typename T>
hipError_t launch_rotate_scatter(const T* g1, const T* g2, int ny, int nx, int P, uint64_t seed,
                                 uint64_t r0, int nb, T* p1, T* p2, long long p_stride, hipStream_t s);
template <typename T>
hipError_t launch_zero2(T* p1, T* p2, long long count, hipStream_t s);
template <typename T>
hipError_t launch_welford_bc(const T* w, long long w_stride, int nb, double* M, double* M2,
                             long long count, int r0, hipStream_t s);
// Peaks above thr of nplanes ny x nx planes under an edge rule (counts:
// nplanes long long, overwritten); with a mask (NULL: none) only peaks whose
// pixel and in-field neighbours are observed.
template <typename T>
hipError_t launch_count_peaks_bc(int ny, int nx, int nplanes, int mode, const T* planes,
                                 const unsigned char* mask, double thr, long long* counts,
                                 hipStream_t s);
// Shear of a masked field (count pixels; mask bytes non-zero = observed;
// outputs may be the inputs).
template <typename T>
hipError_t launch_mask_shear(long long count, const T* g1, const T* g2, const unsigned char* mask,
                             T* o1, T* o2, hipStream_t s);
template <typename T>
hipError_t launch_sigma_snr_bc(const double* M2, int R, const T* w_signal, T* sigma, T* snr,
                               long long count, hipStream_t s);

}  // namespace amap

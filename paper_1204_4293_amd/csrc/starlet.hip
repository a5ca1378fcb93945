// Starlet (a trous, B3-spline) decomposition and reconstruction (Sec. 3 and
// eq:splinewl of the paper).  Step j (1-based) smooths c_{j-1} with the taps
// (1,4,6,4,1)/16 at dilation s = 2^(j-1), first along x then along y, with
// periodic indices, and emits w_j = c_{j-1} - c_j.
//
// Scales are processed in stages of one to three, each stage one kernel
// whose workgroups hold a tile of c in LDS and run the row and column passes
// of all its scales there.  A stage starting at dilation d0 reads rows
// y = q + d0*v (one residue q mod d0 per tile): the stage's dilations are
// then 1, 2, 4 sub-rows along y, and d0, 2 d0, 4 d0 pixels along x, where
// the rows stay contiguous so every HBM access is a long row segment.  The
// tile carries a halo of 2 d0 (2^ns - 1) pixels along x and 2 (2^ns - 1)
// sub-rows along y.  Two LDS buffers: the row pass reads A and writes B, the
// column pass reads B and writes A, one barrier after each; wavefronts take
// rows and lanes take pixels, so no index is divided.  Each thread keeps
// c_{j-1} of its own output pixels in registers to form w_j.  The host picks
// per stage the largest scale count whose tile fits twice in LDS with a
// bounded halo overhead; scales whose dilation leaves no such tile use
// per-scale row and column kernels.
//
// Maps (or noise realisations) are spread over gridDim.y.  For noise maps the
// stage writes its detail planes to a scratch stack and a streaming kernel
// merges them into a running mean and sum of squared deviations per pixel
// (Welford's update over the batch, then Chan, Golub & LeVeque's pairwise
// merge in double precision), so no sum of squares of raw values is ever
// formed.
#include <type_traits>

#include "amap_device.h"
#include "amap_launch.h"

namespace amap {

template <typename T>
__device__ __forceinline__ T b3_combine(T a0, T a1, T a2, T a3, T a4) {
    return ((a0 + a4) + (T)4 * (a1 + a3) + (T)6 * a2) * (T)0.0625;
}

constexpr int kPx = 8;           // output pixels owned per thread
constexpr int kLdsBytes = 160 * 1024 - 1024;

template <typename T>
struct StageArgs {
    int logn, j0, ns;            // scales j0 .. j0+ns-1 (1-based), ns <= 3
    int log_tw, th;              // output tile: 2^log_tw pixels x th sub-rows
    const T* src;                // c_{j0-1} of map blockIdx.y at src + map*src_stride
    long long src_stride;
    T* planes;                   // w_j at planes + map*planes_stride + (j-1-plane_base) n^2
    long long planes_stride;
    int plane_base;
    T* cout;                     // c_{j0+ns-1}, or null
    long long cout_stride;
};

template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_starlet_stage(StageArgs<T> a) {
    extern __shared__ unsigned char smem_raw[];
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = 1 << a.logn, m = n - 1;
    const long long n2 = (long long)n * n;
    const int tw = 1 << a.log_tw, twm = tw - 1;
    const int d0 = 1 << (a.j0 - 1);
    const int Hx = 2 * d0 * ((1 << a.ns) - 1);
    const int Hv = 2 * ((1 << a.ns) - 1);
    const int TXT = tw + 2 * Hx, TVT = a.th + 2 * Hv;
    T* A = reinterpret_cast<T*>(smem_raw);
    T* Bf = A + TXT * TVT;
    // tile index: x-tiles fastest, then sub-row tiles, then the row residue;
    // consecutive tiles (which share halos) are kept on one XCD
    const int ntx = n >> a.log_tw, ntv = (n / d0) / a.th;
    const int ntiles = ntx * ntv * d0;
    int t = blockIdx.x;
    if ((ntiles & 7) == 0) t = (t & 7) * (ntiles >> 3) + (t >> 3);
    const int xt = t % ntx, vt = (t / ntx) % ntv, q = t / (ntx * ntv);
    const int x0 = xt * tw, v0 = vt * a.th;
    const int npix = tw * a.th;
    const int map = blockIdx.y;
    const T* src = a.src + (long long)map * a.src_stride;

    // load the tile with its halo (periodic), one wavefront per row
    for (int v = wave; v < TVT; v += NW) {
        const long long row = (long long)((q + d0 * (v0 - Hv + v)) & m) * n;
        for (int i = lane; i < TXT; i += 64) A[v * TXT + i] = src[row + ((x0 - Hx + i) & m)];
    }
    __syncthreads();

    // c_{j-1} of the owned output pixels, carried from scale to scale
    T prev[kPx];
#pragma unroll
    for (int k = 0; k < kPx; ++k) {
        const int p = tid + k * NT;
        if (p < npix) prev[k] = A[(Hv + (p >> a.log_tw)) * TXT + Hx + (p & twm)];
    }
    int xlo = 0, xhi = TXT, vlo = 0, vhi = TVT;
    for (int s = 0; s < a.ns; ++s) {
        const int dx = d0 << s, dv = 1 << s;
        // row pass A -> B over rows [vlo, vhi), pixels [rlo, rhi)
        const int rlo = xlo + 2 * dx, rhi = xhi - 2 * dx;
        for (int v = vlo + wave; v < vhi; v += NW) {
            const T* ra = A + v * TXT;
            T* rb = Bf + v * TXT;
            for (int i = rlo + lane; i < rhi; i += 64)
                rb[i] = b3_combine(ra[i - 2 * dx], ra[i - dx], ra[i], ra[i + dx], ra[i + 2 * dx]);
        }
        __syncthreads();
        // column pass B -> A over rows [clo, chi), pixels [rlo, rhi)
        const int clo = vlo + 2 * dv, chi = vhi - 2 * dv;
        for (int v = clo + wave; v < chi; v += NW) {
            const T* c0 = Bf + (v - 2 * dv) * TXT;
            const int st = dv * TXT;
            T* ra = A + v * TXT;
            for (int i = rlo + lane; i < rhi; i += 64)
                ra[i] = b3_combine(c0[i], c0[i + st], c0[i + 2 * st], c0[i + 3 * st], c0[i + 4 * st]);
        }
        __syncthreads();
        // w_j of the owned pixels (the next row pass only reads A)
        T* wplane = a.planes + (long long)map * a.planes_stride +
                    (long long)(a.j0 + s - 1 - a.plane_base) * n2;
#pragma unroll
        for (int k = 0; k < kPx; ++k) {
            const int p = tid + k * NT;
            if (p < npix) {
                const int pv = p >> a.log_tw, px = p & twm;
                const T c = A[(Hv + pv) * TXT + Hx + px];
                wplane[(long long)((q + d0 * (v0 + pv)) & m) * n + x0 + px] = prev[k] - c;
                prev[k] = c;
            }
        }
        xlo = rlo; xhi = rhi; vlo = clo; vhi = chi;
    }
    if (a.cout) {
        T* co = a.cout + (long long)map * a.cout_stride;
#pragma unroll
        for (int k = 0; k < kPx; ++k) {
            const int p = tid + k * NT;
            if (p < npix) {
                const int pv = p >> a.log_tw, px = p & twm;
                co[(long long)((q + d0 * (v0 + pv)) & m) * n + x0 + px] = prev[k];
            }
        }
    }
}

// Running per-pixel statistics of noise detail planes.  For each of ns
// scales, the batch of realisations (w at + b*w_map_stride + s*n^2) is
// reduced with Welford's update and merged into the double-precision
// running mean M and sum of squared deviations M2 of the `done`
// realisations before it (pairwise update).  Deterministic: each pixel is
// owned by one thread and realisations are taken in order.
template <typename T>
__global__ void __launch_bounds__(256)
k_welford_merge(const T* __restrict__ w, long long w_map_stride, int ns, int batch, int done,
                long long n2, double* __restrict__ M, double* __restrict__ M2) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n2) return;
    const double na = (double)done, nb = (double)batch, nt = na + nb;
    for (int s = 0; s < ns; ++s) {
        const T* ws = w + (long long)s * n2 + idx;
        double mean = 0.0, m2 = 0.0;
        for (int b = 0; b < batch; ++b) {
            const double v = (double)ws[(long long)b * w_map_stride];
            const double d = v - mean;
            mean += d / (double)(b + 1);
            m2 += d * (v - mean);
        }
        const long long e = (long long)s * n2 + idx;
        const double delta = mean - M[e];
        M[e] += delta * (nb / nt);
        M2[e] += m2 + delta * delta * (na * nb / nt);
    }
}

// ---- per-scale kernels for dilations whose tiles do not fit in LDS -----------------
// Row pass: tmp = h_s (x) c along x.  grid (n*n/256, maps)
template <typename T>
__global__ void __launch_bounds__(256)
k_starlet_row(const T* __restrict__ c, long long c_stride, T* __restrict__ tmp, int logn, int s) {
    const int n = 1 << logn, m = n - 1;
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)n * n) return;
    const int x = (int)(idx & m);
    const T* row = c + (long long)blockIdx.y * c_stride + (idx - x);
    tmp[(long long)blockIdx.y * n * n + idx] =
        b3_combine(row[(x - 2 * s) & m], row[(x - s) & m], row[x], row[(x + s) & m],
                   row[(x + 2 * s) & m]);
}

// Column pass: c_j = h_s (x) tmp along y; w_j = c_{j-1} - c_j.  cprev and
// cnext may be the same array (each thread reads its own pixel first).
template <typename T>
__global__ void __launch_bounds__(256)
k_starlet_col(const T* __restrict__ tmp, const T* cprev, long long cprev_stride,
              T* __restrict__ w, long long w_stride, T* cnext, long long cnext_stride, int logn,
              int s) {
    const int n = 1 << logn, m = n - 1;
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)n * n) return;
    const int x = (int)(idx & m);
    const int y = (int)(idx >> logn);
    const T* t = tmp + (long long)blockIdx.y * n * n + x;
    const T cj = b3_combine(t[(long long)((y - 2 * s) & m) * n], t[(long long)((y - s) & m) * n],
                            t[(long long)y * n], t[(long long)((y + s) & m) * n],
                            t[(long long)((y + 2 * s) & m) * n]);
    const T prev = cprev[(long long)blockIdx.y * cprev_stride + idx];
    w[(long long)blockIdx.y * w_stride + idx] = prev - cj;
    cnext[(long long)blockIdx.y * cnext_stride + idx] = cj;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_reconstruct(const T* __restrict__ planes, T* __restrict__ out, int logn, int J) {
    const long long n2 = 1ll << (2 * logn);
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n2) return;
    T v = planes[(long long)(J - 1) * n2 + idx];
    for (int j = 0; j < J - 1; ++j) v += planes[(long long)j * n2 + idx];
    out[idx] = v;
}

// ---- stage geometry ---------------------------------------------------------------------
struct StageGeom {
    int ns, nt, tw, th;
    size_t lds;
};

// Largest tile overhead accepted for a stage (LDS elements per output pixel).
constexpr double kMaxHaloRatio = 2.6;

// Picks the scale count and tile of the stage starting at scale j0 (at most
// `left` scales remain): the largest ns <= 3 with a tile whose two buffers fit
// in LDS and whose halo overhead is bounded; among those, the smallest
// overhead.  Returns false if no tile exists even for one scale.
template <typename T>
static bool pick_stage(int n, int j0, int left, StageGeom* g) {
    const int d0 = 1 << (j0 - 1);
    for (int ns = left < 3 ? left : 3; ns >= 1; --ns) {
        const int Hx = 2 * d0 * ((1 << ns) - 1), Hv = 2 * ((1 << ns) - 1);
        bool found = false;
        StageGeom best{};
        double best_ratio = 0.0;
        for (int tw = 256; tw >= 16; tw /= 2) {
            for (int th = 64; th >= 2; th /= 2) {
                if (tw > n || th > n / d0) continue;
                const int TXT = tw + 2 * Hx, TVT = th + 2 * Hv;
                const size_t lds = 2 * (size_t)TXT * TVT * sizeof(T);
                if (lds > (size_t)kLdsBytes) continue;
                const double ratio = (double)TXT * TVT / ((double)tw * th);
                if (ratio > kMaxHaloRatio && !(ns == 1 && ratio <= 2 * kMaxHaloRatio)) continue;
                int nt = tw * th / kPx;
                nt = nt < 256 ? 256 : (nt > 512 ? 512 : nt);
                if (tw * th > nt * kPx) continue;
                // prefer small overhead, then more workgroups per CU (less LDS)
                if (!found || ratio < best_ratio - 1e-9 ||
                    (ratio < best_ratio + 1e-9 && lds < best.lds)) {
                    best = StageGeom{ns, nt, tw, th, lds};
                    best_ratio = ratio;
                    found = true;
                }
            }
        }
        if (found) {
            *g = best;
            return true;
        }
    }
    return false;
}

template <typename T, int NT>
static hipError_t launch_stage_nt(const StageArgs<T>& a, const StageGeom& g, int maps,
                                  hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_starlet_stage<T, NT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int n = 1 << a.logn;
    const int d0 = 1 << (a.j0 - 1);
    const unsigned tiles = (unsigned)((n / g.tw) * ((n / d0) / g.th) * d0);
    static const char* names[12] = {"starlet_stage_j1", "starlet_stage_j2", "starlet_stage_j3",
                                    "starlet_stage_j4", "starlet_stage_j5", "starlet_stage_j6",
                                    "starlet_stage_j7", "starlet_stage_j8", "starlet_stage_j9",
                                    "starlet_stage_j10", "starlet_stage_j11", "starlet_stage_j12"};
    AMAP_LAUNCH(names[a.j0 - 1 < 12 ? a.j0 - 1 : 11], s,
                k_starlet_stage<T, NT><<<dim3(tiles, maps), NT, g.lds, s>>>(a));
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_stage(const StageArgs<T>& a, const StageGeom& g, int maps, hipStream_t s) {
    switch (g.nt) {
        case 256: return launch_stage_nt<T, 256>(a, g, maps, s);
        case 512: return launch_stage_nt<T, 512>(a, g, maps, s);
        default: return hipErrorInvalidValue;
    }
}

// Per-scale path of one stage: c_in -> (w_j, c_out) through tmp, w_j at
// w + map*w_stride + (j-1-plane_base)*n^2.
template <typename T>
static hipError_t per_scale_stage(int logn, int j0, int ns, int maps, const T* cin,
                                  long long cin_stride, T* cout, long long cout_stride, T* w,
                                  long long w_stride, int plane_base, T* tmp, hipStream_t st) {
    const long long n2 = 1ll << (2 * logn);
    const dim3 grid((unsigned)((n2 + 255) / 256), maps);
    const T* c = cin;
    long long cstride = cin_stride;
    for (int k = 0; k < ns; ++k) {
        const int j = j0 + k, sdil = 1 << (j - 1);
        T* wj = w + (long long)(j - 1 - plane_base) * n2;
        AMAP_LAUNCH("starlet_row", st,
                    k_starlet_row<T><<<grid, 256, 0, st>>>(c, cstride, tmp, logn, sdil));
        AMAP_LAUNCH("starlet_col", st,
                    k_starlet_col<T><<<grid, 256, 0, st>>>(tmp, c, cstride, wj, w_stride, cout,
                                                          cout_stride, logn, sdil));
        c = cout;
        cstride = cout_stride;
    }
    return hipGetLastError();
}

// Stages: scales 1-3 at d0 = 1, 4-6 at d0 = 8, 7-9 at d0 = 64, ...
// The running c alternates between buffers so that no stage writes the
// array it reads; for the signal the last stage lands in the last plane.
// Noise batches write each stage's planes into wbuf ([batch][3][n^2]) and
// merge them into (M, M2) before the next stage.
template <typename T>
hipError_t launch_starlet(const StarletArgs<T>& a) {
    const int n = 1 << a.logn;
    const long long n2 = (long long)n * n;
    const bool acc = a.M != nullptr;
    // plan the stages: (j0, ns, tile) or a per-scale stage (tile.nt == 0)
    struct Stage { int j0, ns; StageGeom g; bool tiled; };
    Stage plan[16];
    int nstages = 0;
    for (int j0 = 1; j0 < a.J; ) {
        StageGeom g{};
        const bool tiled = pick_stage<T>(n, j0, a.J - j0, &g);
        const int ns = tiled ? g.ns : 1;
        plan[nstages++] = Stage{j0, ns, g, tiled};
        j0 += ns;
    }
    T* final_c = acc ? nullptr : a.planes + (long long)(a.J - 1) * n2;
    const long long final_stride = a.planes_stride;
    const T* cur = a.kappa;
    long long cur_stride = a.in_stride;
    for (int gi = 0; gi < nstages; ++gi) {
        const Stage& st = plan[gi];
        const bool last = gi == nstages - 1;
        T* dst;
        long long dst_stride;
        if (!acc) {
            const int from_end = nstages - 1 - gi;  // the last write lands in final_c
            dst = (from_end % 2 == 0) ? final_c : a.cbuf0;
            dst_stride = (from_end % 2 == 0) ? final_stride : n2;
        } else {
            dst = last ? nullptr : (cur == a.cbuf0 ? a.cbuf1 : a.cbuf0);
            dst_stride = n2;
        }
        // detail planes of this stage
        T* wdst = acc ? a.wbuf : a.planes;
        const long long wstride = acc ? 3 * n2 : a.planes_stride;
        const int pbase = acc ? st.j0 - 1 : 0;
        hipError_t e;
        if (st.tiled) {
            StageArgs<T> s;
            int lt = 0;
            while ((1 << lt) < st.g.tw) ++lt;
            s.logn = a.logn; s.j0 = st.j0; s.ns = st.ns; s.log_tw = lt; s.th = st.g.th;
            s.src = cur; s.src_stride = cur_stride;
            s.planes = wdst; s.planes_stride = wstride; s.plane_base = pbase;
            s.cout = dst; s.cout_stride = dst_stride;
            e = launch_stage<T>(s, st.g, a.batch, a.stream);
        } else {
            // the per-scale path carries c through a buffer even for the last stage
            T* d = dst ? dst : (cur == a.cbuf0 ? a.cbuf1 : a.cbuf0);
            e = per_scale_stage<T>(a.logn, st.j0, st.ns, a.batch, cur, cur_stride, d,
                                   dst ? dst_stride : n2, wdst, wstride, pbase, a.tmp, a.stream);
        }
        if (e != hipSuccess) return e;
        if (acc) {
            AMAP_LAUNCH("welford_merge", a.stream,
                        k_welford_merge<T><<<(unsigned)((n2 + 255) / 256), 256, 0, a.stream>>>(
                            a.wbuf, 3 * n2, st.ns, a.batch, a.done, n2,
                            a.M + (long long)(st.j0 - 1) * n2, a.M2 + (long long)(st.j0 - 1) * n2));
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        cur = dst;
        cur_stride = dst_stride;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reconstruct(int logn, int J, const T* planes, T* out, hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    AMAP_LAUNCH("reconstruct", s,
                k_reconstruct<T><<<(unsigned)((n2 + 255) / 256), 256, 0, s>>>(planes, out, logn, J));
    return hipGetLastError();
}

template hipError_t launch_starlet<float>(const StarletArgs<float>&);
template hipError_t launch_starlet<double>(const StarletArgs<double>&);
template hipError_t launch_reconstruct<float>(int, int, const float*, float*, hipStream_t);
template hipError_t launch_reconstruct<double>(int, int, const double*, double*, hipStream_t);

}  // namespace amap

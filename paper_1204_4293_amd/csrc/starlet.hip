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
// column pass reads B and writes A, one barrier after each; the column pass
// slides a window of five rows down each vector column.  Each thread keeps
// c_{j-1} of its own output pixels in registers to form w_j.  The host picks
// per stage the largest scale count whose tile fits twice in LDS with a
// bounded halo overhead; scales whose dilation leaves no such tile use
// per-scale row and column kernels.
//
// Noise statistics have two more stage kinds, for the coarse scales: tile
// stages on the periodic sub-grid images of d0 (from scale j0 every tap
// joins pixels congruent mod d0, so each sub-grid is a map of its own with
// the dilations of a first stage), and a final stage on whole sub-grids
// held in LDS.
//
// Maps (or noise realisations) are spread over gridDim.y.  For noise maps the
// stages keep a running mean and sum of squared deviations per pixel
// (Welford's update over the batch, then Chan, Golub & LeVeque's pairwise
// merge in double precision), so no sum of squares of raw values is ever
// formed: with few realisations a pixel's spread can be far below its mean,
// and S2 - S1^2 / n would then lose most of its digits.
#include <type_traits>

#include "amap_device.h"
#include "amap_launch.h"

namespace amap {

template <typename T>
__device__ __forceinline__ T b3_combine(T a0, T a1, T a2, T a3, T a4) {
    return ((a0 + a4) + (T)4 * (a1 + a3) + (T)6 * a2) * (T)0.0625;
}
// The tiled passes split the normalisation: a row pass stores 16 times its
// B3 average (b3_row, no multiply) and the column pass scales its sum of
// those by 1/256 (b3_col).  Every factor is a power of two, so each value a
// column pass stores is bit for bit what two normalised passes give.
template <typename T>
__device__ __forceinline__ T b3_row(T a0, T a1, T a2, T a3, T a4) {
    return (a0 + a4) + (T)4 * (a1 + a3) + (T)6 * a2;
}
template <typename T>
__device__ __forceinline__ T b3_col(T a0, T a1, T a2, T a3, T a4) {
    return ((a0 + a4) + (T)4 * (a1 + a3) + (T)6 * a2) * (T)0.00390625;
}

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
    // grouped maps (null: the strided addressing above): map m reads
    // src + src_off[m] and writes its planes at planes + planes_off[m]
    // (element offsets); cout_plane >= 0 puts c_{j0+ns-1} in that plane of
    // the map's planes instead of cout
    const long long* src_off = nullptr;
    const long long* planes_off = nullptr;
    int cout_plane = -1;
};

// 16-byte vectors: four floats or two doubles
template <typename T> struct Vec;
template <> struct Vec<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int G = 4;
};
template <> struct Vec<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int G = 2;
};

template <typename T, int G>
struct VArr { T e[G]; };

// 16-byte loads and stores of G consecutive values (p is 16-byte aligned).
template <typename T, int G>
__device__ __forceinline__ VArr<T, G> vload(const T* p) {
    const typename Vec<T>::type v = *reinterpret_cast<const typename Vec<T>::type*>(p);
    VArr<T, G> r;
#pragma unroll
    for (int c = 0; c < G; ++c) r.e[c] = v[c];
    return r;
}
template <typename T, int G>
__device__ __forceinline__ void vstore(T* p, const VArr<T, G>& r) {
    typename Vec<T>::type v;
#pragma unroll
    for (int c = 0; c < G; ++c) v[c] = r.e[c];
    *reinterpret_cast<typename Vec<T>::type*>(p) = v;
}
// The same store marked non-temporal, for coarse planes that the next stage
// reads back from memory (keeps them from displacing cached inputs).
template <typename T, int G>
__device__ __forceinline__ void vstore_stream(T* p, const VArr<T, G>& r) {
    typename Vec<T>::type v;
#pragma unroll
    for (int c = 0; c < G; ++c) v[c] = r.e[c];
    __builtin_nontemporal_store(v, reinterpret_cast<typename Vec<T>::type*>(p));
}
template <typename T, int G>
__device__ __forceinline__ VArr<T, G> vrow(const VArr<T, G>& a0, const VArr<T, G>& a1,
                                           const VArr<T, G>& a2, const VArr<T, G>& a3,
                                           const VArr<T, G>& a4) {
    VArr<T, G> r;
#pragma unroll
    for (int c = 0; c < G; ++c) r.e[c] = b3_row(a0.e[c], a1.e[c], a2.e[c], a3.e[c], a4.e[c]);
    return r;
}
template <typename T, int G>
__device__ __forceinline__ VArr<T, G> vcol(const VArr<T, G>& a0, const VArr<T, G>& a1,
                                           const VArr<T, G>& a2, const VArr<T, G>& a3,
                                           const VArr<T, G>& a4) {
    VArr<T, G> r;
#pragma unroll
    for (int c = 0; c < G; ++c) r.e[c] = b3_col(a0.e[c], a1.e[c], a2.e[c], a3.e[c], a4.e[c]);
    return r;
}

// Whether the passes can be laid out as a grid over NT threads (as
// tile_scale_pass_grid does) for a tile TXT values wide and a stage of ns
// scales: a tile row's vectors, padded to a multiple of eight, fit the
// threads, and the row groups that leaves cover the dilation 2^(ns-1) of the
// stage's last column pass (its window chains go to row groups in
// multiples of the dilation).
__host__ __device__ constexpr bool grid_fits(int TXT, int G, int NT, int ns) {
    return ((TXT / G + 7) & ~7) <= NT && NT / ((TXT / G + 7) & ~7) >= (1 << (ns - 1));
}

// Geometry shared by the host planner and the kernel: the x halo is rounded
// up to whole vectors so the output tile starts on a vector boundary; each
// LDS row has one vector of padding on either side (read only by outputs
// outside the valid region).
__host__ __device__ inline int stage_hx(int d0, int ns, int G) {
    const int h = 2 * d0 * ((1 << ns) - 1);
    return (h + G - 1) / G * G;
}

constexpr int kSegLen = 4;        // column-pass outputs per sliding window
constexpr int kVecPerThread = 2;  // owned output vectors per thread

// Noise stages: NT threads, each owning KV output vectors (its Welford state
// lives in registers).  Tiles of up to 1024 vectors run one vector per
// thread (256, 512 or 1024 threads); tiles of 2048 vectors run 512 threads
// with four vectors each, which fits the larger state of one or two scales
// in the 256 registers a thread of a 512-thread workgroup may hold.
struct NoiseCfg { int nt, kv; };
__host__ __device__ constexpr NoiseCfg noise_cfg(int vec) {
    return vec <= 256 ? NoiseCfg{256, 1}
         : vec <= 512 ? NoiseCfg{512, 1}
         : vec <= 1024 ? NoiseCfg{1024, 1}
         : NoiseCfg{512, 4};
}
// Prefetch registers (16-byte vectors) per thread and realisation: a tile's
// vectors may not exceed nt times this.  One-vector stages keep 3 (their
// 128-register budget), or 2 when two realisations are processed at a time;
// four-vector stages hold 8.
__host__ __device__ constexpr int noise_prefetch(int /*nt*/, int kv, int rb = 1) {
    return kv > 1 ? 8 : (rb > 1 ? 2 : 3);
}

// Barrier that orders only LDS accesses, so global loads issued before it
// (the next tile's prefetch) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Geometry of one tile of a stage, shared by the write and noise kernels.
struct TileGeom {
    int n, m, d0, Hx, Hv, TXT, TVT, RS, tw, log_tw, th, x0, v0, q, nvec;
    long long base;  // offset of the tile's image in the plane
};

// The tile of this workgroup in a plane that holds 4^logi periodic images
// of side 2^logn one after another (logi = 0: the plane is one image; a
// plane in sub-grid order for d = 2^logi holds its d^2 sub-grids so),
// the stage starting at scale j0 of each image.
__device__ __forceinline__ TileGeom tile_geom(int logn, int j0, int ns, int log_tw, int th,
                                              int G, int logi = 0) {
    TileGeom g;
    g.n = 1 << logn; g.m = g.n - 1;
    g.tw = 1 << log_tw; g.log_tw = log_tw; g.th = th;
    g.d0 = 1 << (j0 - 1);
    g.Hx = stage_hx(g.d0, ns, G);
    g.Hv = 2 * ((1 << ns) - 1);
    g.TXT = g.tw + 2 * g.Hx; g.TVT = th + 2 * g.Hv;
    g.RS = g.TXT + 2 * G;
    // tile index: x-tiles fastest, then sub-row tiles, then the row residue,
    // then the image; consecutive tiles (which share halos) are kept on one XCD
    const int ntx = g.n >> log_tw, ntv = (g.n / g.d0) / th;
    const int ntiles = ntx * ntv * g.d0;
    const int total = ntiles << (2 * logi);
    int t = blockIdx.x;
    if ((total & 7) == 0) t = (t & 7) * (total >> 3) + (t >> 3);
    g.base = 0;
    if (logi > 0) {
        const int img = t / ntiles;
        t -= img * ntiles;
        g.base = (long long)img << (2 * logn);
    }
    const int xt = t % ntx, vt = (t / ntx) % ntv;
    g.q = t / (ntx * ntv);
    g.x0 = xt * g.tw; g.v0 = vt * th;
    g.nvec = (g.tw * th) / G;
    return g;
}

// Offset of tile row v in the plane, and of owned output row pv.
__device__ __forceinline__ long long tile_row(const TileGeom& g, int v) {
    return g.base + (long long)((g.q + g.d0 * (g.v0 - g.Hv + v)) & g.m) * g.n;
}
__device__ __forceinline__ long long out_row(const TileGeom& g, int pv) {
    return g.base + (long long)((g.q + g.d0 * (g.v0 + pv)) & g.m) * g.n;
}

// Splits e into (e / d, e % d) with a float reciprocal; exact for e < 16384
// and d <= 1024 (checked exhaustively on the host).
__device__ __forceinline__ int fdiv(int e, float inv_d) {
    return (int)(((float)e + 0.5f) * inv_d);
}

// Row pass A -> B of one dilation class over rows [vlo, vhi) of each of
// the RB tiles: DXC = 1 or 2 (the five taps of a vector's G outputs lie in
// it and its two neighbours) or 0 (the dilation is a multiple of the vector
// width: five whole-vector taps).  Items are (row, vector) pairs spread over
// all threads; each thread takes U at a time so their LDS reads overlap.
template <typename T, int NT, int RB, int DXC, int U>
__device__ __forceinline__ void row_pass(const T* A, T* Bf, int RS, int dx, int rlo4, int nv,
                                         float inv_nv, int rtot, int vlo, int tstride) {
    constexpr int G = Vec<T>::G;
    using VA = VArr<T, G>;
    // one item: output vector e of the RB tiles' rows (item e of tile t is
    // e + t * rtot), returned with its offset in B
    auto item = [&](int e, VA& o) {
        int tb = 0;
        if (RB > 1 && e >= rtot) { e -= rtot; tb = tstride; }
        const int r = fdiv(e, inv_nv);
        const int i0 = rlo4 + (e - r * nv) * G;
        const int ro = tb + (vlo + r) * RS;
        const T* ra = A + ro;
        if constexpr (DXC != 0) {
            const VA l = vload<T, G>(ra + i0 - G), c = vload<T, G>(ra + i0), rr = vload<T, G>(ra + i0 + G);
            T w[3 * G];
#pragma unroll
            for (int k = 0; k < G; ++k) { w[k] = l.e[k]; w[G + k] = c.e[k]; w[2 * G + k] = rr.e[k]; }
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int b = G + k;  // DXC * 2 <= G keeps every tap inside w
                o.e[k] = b3_row(w[b - 2 * DXC], w[b - DXC], w[b], w[b + DXC], w[b + 2 * DXC]);
            }
        } else {
            o = vrow<T, G>(vload<T, G>(ra + i0 - 2 * dx), vload<T, G>(ra + i0 - dx),
                               vload<T, G>(ra + i0), vload<T, G>(ra + i0 + dx),
                               vload<T, G>(ra + i0 + 2 * dx));
        }
        return ro + i0;
    };
    const int total = RB * rtot;
    for (int e0 = threadIdx.x; e0 < total; e0 += U * NT) {
        VA o[U];
        int off[U];
        if (e0 + (U - 1) * NT < total) {  // all U items exist: no guards
#pragma unroll
            for (int u = 0; u < U; ++u) off[u] = item(e0 + u * NT, o[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) vstore<T, G>(Bf + off[u], o[u]);
            continue;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NT;
            off[u] = e < total ? item(e, o[u]) : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (off[u] >= 0) vstore<T, G>(Bf + off[u], o[u]);
    }
}

// Row and column passes of scale s of a stage on the tile in A (B is
// scratch); on return A holds c_{j0+s} on the shrunken valid region
// [xlo, xhi) x [vlo, vhi), which the call updates.  With RB > 1 the passes
// cover RB tiles laid out tstride elements apart.  U: row items per thread
// and iteration.
template <typename T, int NT, int RB = 1, int U = 2>
__device__ __forceinline__ void tile_scale_pass(T* A, T* Bf, const TileGeom& g, int s, int& xlo,
                                                int& xhi, int& vlo, int& vhi, int tstride = 0) {
    constexpr int G = Vec<T>::G;
    using VA = VArr<T, G>;
    const int tid = threadIdx.x;
    const int RS = g.RS;
    const int dx = g.d0 << s, dv = 1 << s;
    // row pass A -> B over rows [vlo, vhi), outputs [rlo, rhi) widened to
    // whole vectors (the extra outputs stay outside the valid region); the
    // dilation class is uniform, so the branch sits outside the item loop
    const int rlo = xlo + 2 * dx, rhi = xhi - 2 * dx;
    const int rlo4 = rlo / G * G;
    const int nv = (rhi - rlo4 + G - 1) / G;   // vectors per row
    const float inv_nv = 1.0f / (float)nv;
    const int rtot = nv * (vhi - vlo);
    if (dx == 1) {
        row_pass<T, NT, RB, 1, U>(A, Bf, RS, dx, rlo4, nv, inv_nv, rtot, vlo, tstride);
    } else if (2 * dx <= G) {
        if constexpr (G >= 4) row_pass<T, NT, RB, 2, U>(A, Bf, RS, dx, rlo4, nv, inv_nv, rtot, vlo, tstride);
    } else {
        row_pass<T, NT, RB, 0, U>(A, Bf, RS, dx, rlo4, nv, inv_nv, rtot, vlo, tstride);
    }
    lds_barrier();
    // column pass B -> A: windows of kSegLen outputs along each chain
    // v = clo + phase + dv*t, one vector column per item; all window
    // values are read before any output is written
    const int clo = vlo + 2 * dv, chi = vhi - 2 * dv;
    const int lmax = (chi - clo + dv - 1) / dv;
    const int nseg = (lmax + kSegLen - 1) / kSegLen;
    const int items = nv * dv * nseg;
    for (int it0 = tid; it0 < RB * items; it0 += NT) {
        int it = it0, tb = 0;
        if (RB > 1 && it >= items) { it -= items; tb = tstride; }
        const int r = fdiv(it, inv_nv);
        const int i0 = rlo4 + (it - r * nv) * G;
        const int phase = r & (dv - 1), seg = r >> s;
        const int vfirst = clo + phase + dv * (seg * kSegLen);
        if (vfirst >= chi) continue;
        const T* col = Bf + tb + i0;
        VA win[kSegLen + 4];
        if (vfirst + dv * (kSegLen - 1) < chi) {
            // a whole segment: every tap row lies below chi + 2 dv, no guards
            const int step = dv * RS;
            const T* wp = col + (vfirst - 2 * dv) * RS;
#pragma unroll
            for (int k = 0; k < kSegLen + 4; ++k) win[k] = vload<T, G>(wp + k * step);
            T* op = A + tb + vfirst * RS + i0;
#pragma unroll
            for (int k = 0; k < kSegLen; ++k)
                vstore<T, G>(op + k * step, vcol<T, G>(win[k], win[k + 1], win[k + 2], win[k + 3], win[k + 4]));
            continue;
        }
#pragma unroll
        for (int k = 0; k < kSegLen + 4; ++k) {
            const int v = vfirst + dv * (k - 2);
            if (k < 4 || v < chi + 2 * dv) win[k] = vload<T, G>(col + v * RS);
        }
#pragma unroll
        for (int k = 0; k < kSegLen; ++k) {
            const int v = vfirst + dv * k;
            if (v < chi)
                vstore<T, G>(A + tb + v * RS + i0,
                             vcol<T, G>(win[k], win[k + 1], win[k + 2], win[k + 3], win[k + 4]));
        }
    }
    lds_barrier();
    xlo = rlo; xhi = rhi; vlo = clo; vhi = chi;
}

// Row pass A -> B of one dilation class for the noise stages: the nv
// vectors of a row go to nv consecutive threads and the threads' row groups
// (nrg of them) step down rows [0, nrows) of the pass, so a thread's items
// lie at a fixed stride from its first one at `off`; every item is done for
// each of the RB tiles (tstride apart).
// DXC > 0: the five taps lie in three vectors (dilation DXC <= G / 2);
// DXC = 0: five vector loads at the dilation dx.
template <typename T, int RB, int DXC>
__device__ __forceinline__ void row_pass_grid(const T* A, T* Bf, int off, int r, int nrows, int nrg,
                                              int RS, int dx, int tstride) {
    constexpr int G = Vec<T>::G;
    using VA = VArr<T, G>;
    const int step = nrg * RS;
    // per tile the item's offset, moved by one step per item; the reads are
    // addressed from the leftmost tap vector, so every tap is a non-negative
    // constant offset from one base
    const int lead = DXC > 0 ? G : 2 * dx;
    int ro[RB];  // element offsets (kept as integers: the pointers stay in LDS)
#pragma unroll
    for (int t = 0; t < RB; ++t) ro[t] = t * tstride + off;
    for (; r < nrows; r += nrg) {
        VA o[RB];
#pragma unroll
        for (int t = 0; t < RB; ++t) {
            const T* ra = A + (ro[t] - lead);
            if constexpr (DXC > 0) {
                const VA l = vload<T, G>(ra), c = vload<T, G>(ra + G), rr = vload<T, G>(ra + 2 * G);
                T w[3 * G];
#pragma unroll
                for (int k = 0; k < G; ++k) { w[k] = l.e[k]; w[G + k] = c.e[k]; w[2 * G + k] = rr.e[k]; }
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const int b = G + k;  // DXC * 2 <= G keeps every tap inside w
                    o[t].e[k] = b3_row(w[b - 2 * DXC], w[b - DXC], w[b], w[b + DXC], w[b + 2 * DXC]);
                }
            } else {
                o[t] = vrow<T, G>(vload<T, G>(ra), vload<T, G>(ra + dx), vload<T, G>(ra + 2 * dx),
                                      vload<T, G>(ra + 3 * dx), vload<T, G>(ra + 4 * dx));
            }
        }
#pragma unroll
        for (int t = 0; t < RB; ++t) {
            vstore<T, G>(Bf + ro[t], o[t]);
            ro[t] += step;
        }
    }
}

// Row and column passes of scale s of a noise stage on the RB tiles in A
// (B is scratch), as tile_scale_pass computes them, with the items laid
// out as a grid over the threads: in the row pass thread (rg, col) takes
// vector col of rows rg, rg + nrg, ...; in the column pass window chains
// q = rg, rg + nq, ... of vector column col, nq a multiple of the dilation
// so that a thread's chains share one phase.  Per item only a constant
// stride is added, instead of splitting an item index.
template <typename T, int NT, int RB>
__device__ __forceinline__ void tile_scale_pass_grid(T* A, T* Bf, const TileGeom& g, int s, int& xlo,
                                                     int& xhi, int& vlo, int& vhi, int tstride) {
    constexpr int G = Vec<T>::G;
    using VA = VArr<T, G>;
    const int tid = threadIdx.x;
    const int RS = g.RS;
    const int dx = g.d0 << s, dv = 1 << s;
    const int rlo = xlo + 2 * dx, rhi = xhi - 2 * dx;
    const int rlo4 = rlo / G * G;
    const int nv = (rhi - rlo4 + G - 1) / G;   // vectors per row, <= TXT / G <= NT (host-checked)
    // a row's vectors go to a multiple of 8 lanes, so that every group of
    // eight lanes (one 128-byte LDS access) stays inside one row
    const int nvp = (nv + 7) & ~7;
    const int rg = fdiv(tid, 1.0f / (float)nvp);
    const int col = tid - rg * nvp;
    const int nrg = NT / nvp;
    const int xoff = rlo4 + col * G;
    if (rg < nrg && col < nv) {
        const int off = (vlo + rg) * RS + xoff;
        const int nrows = vhi - vlo;
        if (dx == 1) {
            row_pass_grid<T, RB, 1>(A, Bf, off, rg, nrows, nrg, RS, dx, tstride);
        } else if (2 * dx <= G) {
            if constexpr (G >= 4) row_pass_grid<T, RB, 2>(A, Bf, off, rg, nrows, nrg, RS, dx, tstride);
        } else {
            row_pass_grid<T, RB, 0>(A, Bf, off, rg, nrows, nrg, RS, dx, tstride);
        }
    }
    lds_barrier();
    const int clo = vlo + 2 * dv, chi = vhi - 2 * dv;
    const int lmax = (chi - clo + dv - 1) / dv;
    const int nseg = (lmax + kSegLen - 1) / kSegLen;
    const int nchain = dv * nseg;            // window chains per vector column and tile
    const int nq = nrg & ~(dv - 1);          // chains in flight per column, a multiple of dv
    if (rg < nq && col < nv) {
        // chain q of the RB tiles' RB * nchain: tile q / nchain, phase q mod dv
        const int phase = rg & (dv - 1);
        const int step = dv * RS;
        for (int q = rg; q < RB * nchain; q += nq) {
            int qq = q, tb = 0;
            if (RB > 1 && qq >= nchain) { qq -= nchain; tb = tstride; }
            const int vfirst = clo + phase + dv * ((qq >> s) * kSegLen);
            if (vfirst >= chi) continue;
            const T* wp = Bf + tb + xoff + (vfirst - 2 * dv) * RS;
            T* op = A + tb + xoff + vfirst * RS;
            VA win[kSegLen + 4];
            if (vfirst + dv * (kSegLen - 1) < chi) {  // a whole segment
#pragma unroll
                for (int k = 0; k < kSegLen + 4; ++k) win[k] = vload<T, G>(wp + k * step);
#pragma unroll
                for (int k = 0; k < kSegLen; ++k)
                    vstore<T, G>(op + k * step, vcol<T, G>(win[k], win[k + 1], win[k + 2], win[k + 3], win[k + 4]));
            } else {
#pragma unroll
                for (int k = 0; k < kSegLen + 4; ++k)
                    if (k < 4 || vfirst + dv * (k - 2) < chi + 2 * dv) win[k] = vload<T, G>(wp + k * step);
#pragma unroll
                for (int k = 0; k < kSegLen; ++k)
                    if (vfirst + dv * k < chi)
                        vstore<T, G>(op + k * step, vcol<T, G>(win[k], win[k + 1], win[k + 2], win[k + 3], win[k + 4]));
            }
        }
    }
    lds_barrier();
    xlo = rlo; xhi = rhi; vlo = clo; vhi = chi;
}

// Owned vector k of the tile: its LDS offset and global offset in a plane.
__device__ __forceinline__ int owned_lds(const TileGeom& g, int e) {
    return (g.Hv + (e >> g.log_tw)) * g.RS + g.Hx + (e & (g.tw - 1));
}
__device__ __forceinline__ long long owned_global(const TileGeom& g, int e) {
    return out_row(g, e >> g.log_tw) + g.x0 + (e & (g.tw - 1));
}

template <typename T, int NT, int KV>
__device__ __forceinline__ void load_owned(const T* A, const TileGeom& g,
                                           VArr<T, Vec<T>::G> (&prev)[KV]) {
    constexpr int G = Vec<T>::G;
#pragma unroll
    for (int k = 0; k < KV; ++k) {
        const int p = threadIdx.x + k * NT;
        if (p < g.nvec) {
            const int e = p * G;
            prev[k] = vload<T, G>(A + (g.Hv + (e >> g.log_tw)) * g.RS + g.Hx + (e & (g.tw - 1)));
        }
    }
}

template <typename T, int NT, int KV>
__device__ __forceinline__ void store_owned(T* dst, const TileGeom& g,
                                            const VArr<T, Vec<T>::G> (&val)[KV]) {
    constexpr int G = Vec<T>::G;
#pragma unroll
    for (int k = 0; k < KV; ++k) {
        const int p = threadIdx.x + k * NT;
        if (p < g.nvec) {
            const int e = p * G;
            const int pv = e >> g.log_tw, px = e & (g.tw - 1);
            vstore<T, G>(dst + out_row(g, pv) + g.x0 + px, val[k]);
        }
    }
}

// Write mode: maps in gridDim.y; stores w_j and the stage's last c.  The
// planes are written once and not read again here, so they go out with
// non-temporal stores.
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_starlet_stage(StageArgs<T> a) {
    extern __shared__ unsigned char smem_raw[];
    constexpr int G = Vec<T>::G;
    using VA = VArr<T, G>;
    const TileGeom g = tile_geom(a.logn, a.j0, a.ns, a.log_tw, a.th, G);
    const long long n2 = (long long)g.n * g.n;
    T* A = reinterpret_cast<T*>(smem_raw) + G;  // element (v, i) at A[v*RS + i], i in [-G, TXT+G)
    T* Bf = A + g.RS * g.TVT;
    const int map = blockIdx.y;
    const T* src = a.src + (a.src_off ? a.src_off[map] : (long long)map * a.src_stride);
    // the tile (with its halo) into LDS: every thread's vectors at a stride
    // of NT over the tile, four loads in flight before their stores
    const int tvec = g.TXT / G, nload = g.TVT * tvec;
    const float inv_tvec = 1.0f / (float)tvec;
    for (int e0 = threadIdx.x; e0 < nload; e0 += 4 * NT) {
        VA r[4];
        int off[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = e0 + k * NT;
            off[k] = -1;
            if (e < nload) {
                const int v = fdiv(e, inv_tvec), c = e - v * tvec;
                r[k] = vload<T, G>(src + tile_row(g, v) + ((g.x0 - g.Hx + c * G) & g.m));
                off[k] = v * g.RS + c * G;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (off[k] >= 0) vstore<T, G>(A + off[k], r[k]);
    }
    lds_barrier();
    VA prev[kVecPerThread];
    load_owned<T, NT, kVecPerThread>(A, g, prev);
    T* planes = a.planes + (a.planes_off ? a.planes_off[map] : (long long)map * a.planes_stride);
    int xlo = 0, xhi = g.TXT, vlo = 0, vhi = g.TVT;
    for (int s = 0; s < a.ns; ++s) {
        tile_scale_pass<T, NT>(A, Bf, g, s, xlo, xhi, vlo, vhi);
        // w of the owned vectors (the next row pass only reads A)
        T* wp = planes + (long long)(a.j0 + s - 1 - a.plane_base) * n2;
#pragma unroll
        for (int k = 0; k < kVecPerThread; ++k) {
            const int p = threadIdx.x + k * NT;
            if (p < g.nvec) {
                const VA c = vload<T, G>(A + owned_lds(g, p * G));
                VA wv;
#pragma unroll
                for (int cc = 0; cc < G; ++cc) wv.e[cc] = prev[k].e[cc] - c.e[cc];
                vstore_stream<T, G>(wp + owned_global(g, p * G), wv);
                prev[k] = c;
            }
        }
    }
    if (a.cout_plane >= 0)
        store_owned<T, NT, kVecPerThread>(planes + (long long)a.cout_plane * n2, g, prev);
    else if (a.cout)
        store_owned<T, NT, kVecPerThread>(a.cout + (long long)map * a.cout_stride, g, prev);
}

// Noise mode: each workgroup owns one tile and takes the realisations
// b = group, group + groups, ... of the batch in turn, prefetching the next
// realisation's tile into registers while the current one is processed.
// Welford's running mean and sum of squared deviations of every owned pixel
// and scale stay in registers; at the end they are merged (Chan's pairwise
// update, double precision) into M, M2, or, with several groups, written as
// partials that k_merge_partials folds in group order.
template <typename T>
struct NoiseStageArgs {
    int logn, j0, ns, log_tw, th;
    const T* src;            // c_{j0-1} of realisation b at src + b*n^2
    T* cout;                 // c_{j0+ns-1} of realisation b at cout + b*n^2, or null
    int batch, groups, done;
    double* M;               // [ns][n^2] running totals of the stage's scales
    double* M2;
    void* part;              // [groups][ns][2][n^2] partials (accumulator type) when groups > 1
    float inv_tvec;          // 1 / (vectors per tile row), for index splitting
    int cout_logd = 0;       // > 0: cout in sub-grid order for d = 2^cout_logd (subgrid_index),
                             // within each image
    int img_logd = 0;        // > 0: src, cout, M and M2 hold the d^2 sub-grids of d = 2^img_logd
                             // (subgrid_index) as periodic images, each transformed on its own
};

// Single-precision one-vector stages of 256 or 512 threads keep to 128
// registers, so that two or more workgroups share a CU and overlap each
// other's barrier phases.
// SG: the coarse output goes out in sub-grid order (a.cout_logd > 0), a
// separate instantiation so that other stages carry none of its registers.
template <typename T, int NT, int NS, int KV, int RB, bool SG>
__global__ void __launch_bounds__(NT, (sizeof(T) == 4 && KV == 1 && NT <= 512) ? 4 : 1)
k_starlet_noise_stage(NoiseStageArgs<T> a) {
    extern __shared__ unsigned char smem_raw[];
    constexpr int G = Vec<T>::G;
    using VA = VArr<T, G>;
    using AccT = typename std::conditional<sizeof(T) == 8, double, float>::type;
    // on sub-grid images, scale j0 is the image's scale j0 - img_logd
    const int logm = a.logn - a.img_logd;
    const TileGeom g = tile_geom(logm, a.j0 - a.img_logd, NS, a.log_tw, a.th, G, a.img_logd);
    const long long n2 = 1ll << (2 * a.logn);
    // RB realisations at a time, tile t in [A_t | B_t], A_t = A + t * tstride
    const int tstride = 2 * g.RS * g.TVT;
    T* A = reinterpret_cast<T*>(smem_raw) + G;
    T* Bf = A + g.RS * g.TVT;
    const int grp = blockIdx.y;
    const int count = (a.batch - grp + a.groups - 1) / a.groups;
    const int rounds = (count + RB - 1) / RB;
    const int tvec = g.TXT / G;
    const int nload = tvec * g.TVT;

    constexpr int PF = noise_prefetch(NT, KV, RB);
    VA pf[RB][PF];
    AccT mean[NS][KV][G], m2[NS][KV][G];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int k = 0; k < KV; ++k)
#pragma unroll
            for (int c = 0; c < G; ++c) mean[s][k][c] = m2[s][k][c] = (AccT)0;
    // owned vectors threadIdx.x + k*NT, k < KV
    bool owner[KV];
    int own_e[KV];
#pragma unroll
    for (int k = 0; k < KV; ++k) {
        owner[k] = (int)threadIdx.x + k * NT < g.nvec;
        own_e[k] = ((int)threadIdx.x + k * NT) * G;
    }
    // tile of the i-th realisation of this group into prefetch slot t
    auto fetch = [&](int i, int t) {
        const T* src = a.src + (long long)(grp + i * a.groups) * n2;
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < nload) {
                const int v = fdiv(e, a.inv_tvec);
                pf[t][k] = vload<T, G>(src + tile_row(g, v) + ((g.x0 - g.Hx + (e - v * tvec) * G) & g.m));
            }
        }
    };

    // the coarse values a round hands on are stored during the next round,
    // before its loads are issued: waiting for a round's loads then never
    // waits for stores issued after them.  Three-scale and four-vector
    // stages have no registers to spare and store at once, and so do stages
    // whose output goes out in sub-grid order (its addresses would spill).
    constexpr bool DEFER = NS < 3 && KV == 1 && !SG;
    VA keep[RB][KV];
    // Sub-grid order of the coarse output (for d = 2^cout_logd): where the
    // tile width is a multiple of G d, a tile row holds, per sub-grid
    // column p, whole vectors of G consecutive sub-grid pixels; the owned
    // vector (row pv, index ix) then stands for vector xg = ix % per of
    // sub-grid column p = ix / per (per = tw / (G d)), gathered from LDS
    // and stored whole.  Otherwise each value is stored on its own.  (Going
    // out sub-grid by sub-grid instead, so that a wavefront writes the rows
    // of one or two sub-grids, measured 15% slower: its strided gathers
    // from LDS conflict in the banks.)
    const int sgd = SG ? 1 << a.cout_logd : 0;
    const bool sg_vec = SG && g.tw % (G * sgd) == 0;
    // the tile row and tile-relative column of that vector's first pixel
    // (every factor is a power of two: shifts and masks only)
    constexpr int LOG_G = G == 4 ? 2 : 1;
    const int lper = g.log_tw - LOG_G - a.cout_logd;  // log2 per
    auto sg_pos = [&](int e, int& pv, int& xr) {
        pv = e >> g.log_tw;
        const int ix = (e & (g.tw - 1)) >> LOG_G;
        xr = (ix >> lper) + ((ix & ((1 << lper) - 1)) << (a.cout_logd + LOG_G));
    };
    auto store_coarse = [&](int i0p) {  // round starting at realisation i0p
#pragma unroll
        for (int t = 0; t < RB; ++t) {
            if (i0p + t >= count) continue;
            const int b = grp + (i0p + t) * a.groups;
#pragma unroll
            for (int k = 0; k < KV; ++k) {
                if (!owner[k]) continue;
                T* dst = a.cout + (long long)b * n2;
                const long long gi = owned_global(g, own_e[k]);
                if constexpr (!SG) {
                    vstore_stream<T, G>(dst + gi, keep[t][k]);
                } else if (sg_vec) {
                    int pv, xr;
                    sg_pos(own_e[k], pv, xr);
                    vstore_stream<T, G>(dst + g.base + subgrid_index(out_row(g, pv) - g.base + g.x0 + xr,
                                                                     logm, a.cout_logd),
                                        keep[t][k]);
                } else {
#pragma unroll
                    for (int c = 0; c < G; ++c)
                        dst[g.base + subgrid_index(gi - g.base + c, logm, a.cout_logd)] = keep[t][k].e[c];
                }
            }
        }
    };

#pragma unroll
    for (int t = 0; t < RB; ++t)
        if (t < count) fetch(t, t);
    for (int ro = 0; ro < rounds; ++ro) {
        const int i0 = ro * RB;  // first realisation index of the round
        lds_barrier();  // the previous round is done with the tiles
        // all of this round's loads are needed below; waiting for every
        // outstanding memory operation here leaves none pending, so the
        // loads issued next are not serialised behind conservative waits
        __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
        for (int t = 0; t < RB; ++t) {
            if (i0 + t >= count) continue;
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                const int e = threadIdx.x + k * NT;
                if (e < nload) {
                    const int v = fdiv(e, a.inv_tvec);
                    vstore<T, G>(A + t * tstride + v * g.RS + (e - v * tvec) * G, pf[t][k]);
                }
            }
        }
        if (DEFER && a.cout && ro > 0) store_coarse(i0 - RB);
#pragma unroll
        for (int t = 0; t < RB; ++t)  // prefetch the next round's tiles
            if (i0 + RB + t < count) fetch(i0 + RB + t, t);
        lds_barrier();
        VA prev[RB][KV];
#pragma unroll
        for (int t = 0; t < RB; ++t)
#pragma unroll
            for (int k = 0; k < KV; ++k)
                if (owner[k]) prev[t][k] = vload<T, G>(A + t * tstride + owned_lds(g, own_e[k]));
        int xlo = 0, xhi = g.TXT, vlo = 0, vhi = g.TVT;
        // Welford weights 1 / (number of realisations so far), once per round
        AccT inv[RB];
#pragma unroll
        for (int t = 0; t < RB; ++t) inv[t] = (AccT)1 / (AccT)(i0 + t + 1);
#pragma unroll
        for (int s = 0; s < NS; ++s) {  // unrolled: the Welford state keeps static indices
            // three scales of sums leave no registers for a second row item
            tile_scale_pass_grid<T, NT, RB>(A, Bf, g, s, xlo, xhi, vlo, vhi, tstride);
            // realisations in order, so the update sequence matches one at a time
#pragma unroll
            for (int t = 0; t < RB; ++t) {
                if (i0 + t >= count) continue;
#pragma unroll
                for (int k = 0; k < KV; ++k) {
                    if (!owner[k]) continue;
                    const VA c = vload<T, G>(A + t * tstride + owned_lds(g, own_e[k]));
#pragma unroll
                    for (int cc = 0; cc < G; ++cc) {
                        const AccT x = (AccT)(prev[t][k].e[cc] - c.e[cc]);
                        const AccT d = x - mean[s][k][cc];
                        mean[s][k][cc] = fma(d, inv[t], mean[s][k][cc]);
                        m2[s][k][cc] = fma(d, x - mean[s][k][cc], m2[s][k][cc]);
                    }
                    prev[t][k] = c;
                }
            }
        }
        if (a.cout) {
#pragma unroll
            for (int t = 0; t < RB; ++t)
#pragma unroll
                for (int k = 0; k < KV; ++k) {
                    if (SG && sg_vec && owner[k]) {  // the tile is complete in LDS since the last barrier
                        int pv, xr;
                        sg_pos(own_e[k], pv, xr);
                        const T* src = A + t * tstride + (g.Hv + pv) * g.RS + g.Hx + xr;
#pragma unroll
                        for (int c = 0; c < G; ++c) keep[t][k].e[c] = src[sgd * c];
                    } else {
                        keep[t][k] = prev[t][k];
                    }
                }
            if (!DEFER) store_coarse(i0);
        }
    }
    if (DEFER && a.cout && rounds > 0) store_coarse((rounds - 1) * RB);
    // merge into the running totals (all loads first: M and M2 do not
    // overlap), or leave partials per group
    if (a.groups == 1) {
        const double na = (double)a.done, nb = (double)count, nt = na + nb;
        const double fb = nb / nt, fab = na * nb / nt;
        double* __restrict__ Mp = a.M;
        double* __restrict__ Qp = a.M2;
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            if (!owner[k]) continue;
            const long long base = owned_global(g, own_e[k]);  // a multiple of G
            double2 mo[NS][G / 2], qo[NS][G / 2];
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int h = 0; h < G / 2; ++h) {
                    if (a.done == 0) {  // the first batch: nothing merged yet, M and M2 unread
                        mo[s][h] = make_double2(0.0, 0.0);
                        qo[s][h] = make_double2(0.0, 0.0);
                    } else {
                        mo[s][h] = *reinterpret_cast<const double2*>(Mp + s * n2 + base + 2 * h);
                        qo[s][h] = *reinterpret_cast<const double2*>(Qp + s * n2 + base + 2 * h);
                    }
                }
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int h = 0; h < G / 2; ++h) {
                    const double d0 = (double)mean[s][k][2 * h] - mo[s][h].x;
                    const double d1 = (double)mean[s][k][2 * h + 1] - mo[s][h].y;
                    mo[s][h].x += d0 * fb;
                    mo[s][h].y += d1 * fb;
                    qo[s][h].x += (double)m2[s][k][2 * h] + d0 * d0 * fab;
                    qo[s][h].y += (double)m2[s][k][2 * h + 1] + d1 * d1 * fab;
                    *reinterpret_cast<double2*>(Mp + s * n2 + base + 2 * h) = mo[s][h];
                    *reinterpret_cast<double2*>(Qp + s * n2 + base + 2 * h) = qo[s][h];
                }
        }
    } else {
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            if (!owner[k]) continue;
            const long long base = owned_global(g, own_e[k]);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                AccT* pp = static_cast<AccT*>(a.part) + ((long long)grp * NS + s) * 2 * n2;
#pragma unroll
                for (int c = 0; c < G; ++c) {
                    pp[base + c] = mean[s][k][c];
                    pp[n2 + base + c] = m2[s][k][c];
                }
            }
        }
    }
}

// Noise mode, final stage on whole sub-grids.  From scale j0 on, with
// d0 = 2^(j0-1), every tap of every remaining scale stays inside one
// sub-grid of d0 (subgrid_index): scale j0 + s is the same B3 cascade on the
// m x m periodic sub-grid at dilation 2^s.  A workgroup holds one sub-grid
// in LDS, so there is no halo and the wrap is an index mask; each thread
// owns one vector, computes it in both passes of every scale and keeps its
// Welford state (same update as the tile stages) in registers.  src holds
// c_{j0-1} of realisation b at src + b n^2 in sub-grid order, M and M2 the
// stage's planes in sub-grid order.  Grid (d0^2 sub-grids, groups).
template <typename T>
struct NoiseSubArgs {
    int logn, j0;
    const T* src;
    int batch, groups, done;
    double* M;
    double* M2;
    void* part;  // [groups][ns][2][n^2] partials when groups > 1
    int rb;      // realisations per pass (1 or 2)
};

template <typename T, int LOGM, int NS, int RB>
__global__ void __launch_bounds__((1 << (2 * LOGM)) / Vec<T>::G)
k_starlet_noise_subgrid(NoiseSubArgs<T> a) {
    constexpr int G = Vec<T>::G;
    constexpr int M = 1 << LOGM, MV = M / G;   // side, vectors per row
    constexpr int RS = M;  // LDS row stride: unpadded (padding by 1-3 vectors measured 20% slower)
    constexpr int TS = M * RS;                 // LDS tile stride (RB tiles per pass)
    using VA = VArr<T, G>;
    using AccT = typename std::conditional<sizeof(T) == 8, double, float>::type;
    extern __shared__ __align__(16) unsigned char sub_smem[];  // subgrid_lds_bytes
    T* A = reinterpret_cast<T*>(sub_smem);
    T* B = A + RB * TS;
    const long long n2 = 1ll << (2 * a.logn);
    const int grp = blockIdx.y;
    const int count = (a.batch - grp + a.groups - 1) / a.groups;
    const int yo = threadIdx.x / MV, xo = (threadIdx.x % MV) * G;  // the owned vector
    const int own = yo * RS + xo;
    const long long gown = ((long long)blockIdx.x << (2 * LOGM)) + (yo << LOGM) + xo;
    AccT mean[NS][G], m2[NS][G];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int c = 0; c < G; ++c) mean[s][c] = m2[s][c] = (AccT)0;
    auto fetch = [&](int i) {
        const int ii = i < count ? i : count - 1;  // past the end: a harmless reload
        return vload<T, G>(a.src + (long long)(grp + ii * a.groups) * n2 + gown);
    };
    // PD realisations in flight ahead of the pass being transformed
    constexpr int PD = RB == 1 ? 3 : 4;
    VA pf[PD];
    if (count > 0) {
#pragma unroll
        for (int k = 0; k < PD; ++k) pf[k] = fetch(k);
    }
    for (int i0 = 0; i0 < count; i0 += RB) {
        VA prev[RB];
#pragma unroll
        for (int t = 0; t < RB; ++t) prev[t] = pf[t];
#pragma unroll
        for (int k = 0; k + RB < PD; ++k) pf[k] = pf[k + RB];
#pragma unroll
        for (int k = PD - RB; k < PD; ++k) pf[k] = fetch(i0 + k + RB);
#pragma unroll
        for (int t = 0; t < RB; ++t) vstore<T, G>(A + t * TS + own, prev[t]);
        // Welford weights 1 / (number of realisations so far), once per round
        AccT inv[RB];
#pragma unroll
        for (int t = 0; t < RB; ++t) inv[t] = (AccT)1 / (AccT)(i0 + t + 1);
        __syncthreads();  // A complete; every read of B by the previous pass done
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int d = 1 << s;  // dilation in sub-grid units
#pragma unroll
            for (int t = 0; t < RB; ++t) {
                const T* ra = A + t * TS + yo * RS;
                VA o;
                if (2 * d <= G) {  // the five taps of the G outputs lie in three vectors
                    const VA l = vload<T, G>(ra + ((xo - G) & (M - 1))), c = vload<T, G>(ra + xo),
                             r = vload<T, G>(ra + ((xo + G) & (M - 1)));
                    T w[3 * G];
#pragma unroll
                    for (int k = 0; k < G; ++k) { w[k] = l.e[k]; w[G + k] = c.e[k]; w[2 * G + k] = r.e[k]; }
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const int b = G + k;
                        o.e[k] = d == 1 ? b3_row(w[b - 2], w[b - 1], w[b], w[b + 1], w[b + 2])
                                        : b3_row(w[b - 4 > 0 ? b - 4 : 0], w[b - 2], w[b], w[b + 2],
                                                     w[b + 4 < 3 * G ? b + 4 : 3 * G - 1]);
                    }
                } else {  // the dilation is a multiple of the vector width
                    o = vrow<T, G>(vload<T, G>(ra + ((xo - 2 * d) & (M - 1))), vload<T, G>(ra + ((xo - d) & (M - 1))),
                                       vload<T, G>(ra + xo), vload<T, G>(ra + ((xo + d) & (M - 1))),
                                       vload<T, G>(ra + ((xo + 2 * d) & (M - 1))));
                }
                vstore<T, G>(B + t * TS + own, o);
            }
            __syncthreads();  // B complete
            // realisations in order, so the Welford sequence matches one at a time
#pragma unroll
            for (int t = 0; t < RB; ++t) {
                const T* cb = B + t * TS + xo;
                const VA c = vcol<T, G>(vload<T, G>(cb + ((yo - 2 * d) & (M - 1)) * RS),
                                            vload<T, G>(cb + ((yo - d) & (M - 1)) * RS),
                                            vload<T, G>(cb + yo * RS),
                                            vload<T, G>(cb + ((yo + d) & (M - 1)) * RS),
                                            vload<T, G>(cb + ((yo + 2 * d) & (M - 1)) * RS));
                if (RB == 1 || i0 + t < count) {
#pragma unroll
                    for (int cc = 0; cc < G; ++cc) {
                        const AccT x = (AccT)(prev[t].e[cc] - c.e[cc]);
                        const AccT dd = x - mean[s][cc];
                        mean[s][cc] = fma(dd, inv[t], mean[s][cc]);
                        m2[s][cc] = fma(dd, x - mean[s][cc], m2[s][cc]);
                    }
                }
                prev[t] = c;
                if (s + 1 < NS) vstore<T, G>(A + t * TS + own, c);  // A's row-pass reads ended at the barrier
            }
            if (s + 1 < NS) __syncthreads();  // A complete; every read of B done
        }
    }
    // merge into the running totals, or leave partials per group
    if (a.groups == 1) {
        const double na = (double)a.done, nb = (double)count, nt = na + nb;
        const double fb = nb / nt, fab = na * nb / nt;
        double* __restrict__ Mp = a.M;
        double* __restrict__ Qp = a.M2;
        double mo[NS][G], qo[NS][G];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < G; ++c) {
                mo[s][c] = a.done == 0 ? 0.0 : Mp[s * n2 + gown + c];  // the first batch: unread
                qo[s][c] = a.done == 0 ? 0.0 : Qp[s * n2 + gown + c];
            }
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < G; ++c) {
                const double dl = (double)mean[s][c] - mo[s][c];
                Mp[s * n2 + gown + c] = mo[s][c] + dl * fb;
                Qp[s * n2 + gown + c] = qo[s][c] + ((double)m2[s][c] + dl * dl * fab);
            }
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            AccT* pp = static_cast<AccT*>(a.part) + ((long long)grp * NS + s) * 2 * n2;
#pragma unroll
            for (int c = 0; c < G; ++c) {
                pp[gown + c] = mean[s][c];
                pp[n2 + gown + c] = m2[s][c];
            }
        }
    }
}

// Folds the per-group partials of one batch, in group order, into M, M2.
template <typename P>
__global__ void __launch_bounds__(256)
k_merge_partials(const P* __restrict__ part, int groups, int ns, int batch, int done,
                 long long n2, double* __restrict__ M, double* __restrict__ M2) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n2) return;
    for (int s = 0; s < ns; ++s) {
        double na = (double)done;
        double mean = done == 0 ? 0.0 : M[(long long)s * n2 + idx];  // the first batch: unread
        double m2 = done == 0 ? 0.0 : M2[(long long)s * n2 + idx];
        for (int grp = 0; grp < groups; ++grp) {
            const double nb = (double)((batch - grp + groups - 1) / groups);
            if (nb == 0.0) continue;
            const P* pp = part + ((long long)grp * ns + s) * 2 * n2;
            const double mb = (double)pp[idx], qb = (double)pp[n2 + idx];
            const double nt = na + nb, delta = mb - mean;
            mean += delta * (nb / nt);
            m2 += qb + delta * delta * (na * nb / nt);
            na = nt;
        }
        M[(long long)s * n2 + idx] = mean;
        M2[(long long)s * n2 + idx] = m2;
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
        const double mo = done == 0 ? 0.0 : M[e], qo = done == 0 ? 0.0 : M2[e];  // the first batch: unread
        const double delta = mean - mo;
        M[e] = mo + delta * (nb / nt);
        M2[e] = qo + (m2 + delta * delta * (na * nb / nt));
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
    int rb = 1;  // realisations per LDS pass (noise stages)
};

// Most tile candidates of one stage (tile widths x heights x pass widths).
constexpr int kMaxCand = 64;

// Largest tile overhead accepted for a stage (LDS elements per output pixel).
constexpr double kMaxHaloRatio = 2.6;

// Tiles for a stage of ns scales from j0 whose two LDS buffers fit and whose
// halo overhead is bounded, best first (smallest overhead, then least LDS);
// noise stages also need the tile to fit the prefetch registers and one
// owned vector per thread.  Float noise stages of one or two scales with one
// owned vector per thread are also offered with two realisations per LDS
// pass (twice the LDS, fewer barriers per realisation).  Returns the number
// written to out (at most cap).
template <typename T>
static int stage_candidates(int n, int j0, int ns, bool noise, StageGeom* out, int cap) {
    constexpr int G = Vec<T>::G;
    const int d0 = 1 << (j0 - 1);
    const int Hx = stage_hx(d0, ns, G), Hv = 2 * ((1 << ns) - 1);
    StageGeom all[kMaxCand];
    double ratio[kMaxCand];
    int m = 0;
    auto insert = [&](const StageGeom& sg, double r) {  // by (overhead, LDS)
        int k = m++;
        while (k > 0 && (r < ratio[k - 1] - 1e-9 ||
                         (r < ratio[k - 1] + 1e-9 && sg.lds < all[k - 1].lds))) {
            all[k] = all[k - 1];
            ratio[k] = ratio[k - 1];
            --k;
        }
        all[k] = sg;
        ratio[k] = r;
    };
    for (int tw = 256; tw >= 16; tw /= 2) {
        for (int th = 64; th >= 2; th /= 2) {
            if (tw > n || th > n / d0) continue;
            const int TXT = tw + 2 * Hx, TVT = th + 2 * Hv;
            const size_t lds = 2 * (size_t)(TXT + 2 * G) * TVT * sizeof(T) + G * sizeof(T);
            if (lds > (size_t)kLdsBytes) continue;
            const double r = (double)TXT * TVT / ((double)tw * th);
            if (r > kMaxHaloRatio && !(ns == 1 && r <= 2 * kMaxHaloRatio)) continue;
            int nt = tw * th / (G * kVecPerThread);
            nt = nt < 256 ? 256 : (nt > 512 ? 512 : nt);
            if (!noise && tw * th > nt * G * kVecPerThread) continue;  // write kernel: 2 vectors per thread
            if (noise) {
                const int vec = tw * th / G;
                if (vec > 2048) continue;  // owned vectors of at most 512 threads x 4
                const NoiseCfg cfg = noise_cfg(vec);
                if (sizeof(T) == 8 && cfg.nt > 512) continue;  // no 1024-thread double stages
                if (cfg.kv > 1 && ns == 3) continue;  // three scales of state for 4 vectors would spill
                if ((TXT / G) * TVT > cfg.nt * noise_prefetch(cfg.nt, cfg.kv)) continue;
                if (!grid_fits(TXT, G, cfg.nt, ns)) continue;  // a tile row's vectors spread over the threads
            }
            insert(StageGeom{ns, nt, tw, th, lds, 1}, r);
            if (noise && sizeof(T) == 4 && ns <= 2) {
                const NoiseCfg cfg = noise_cfg(tw * th / G);
                const size_t lds2 = 4 * (size_t)(TXT + 2 * G) * TVT * sizeof(T) + G * sizeof(T);
                if (cfg.kv == 1 && lds2 <= (size_t)kLdsBytes &&
                    (TXT / G) * TVT <= cfg.nt * noise_prefetch(cfg.nt, 1, 2))
                    insert(StageGeom{ns, nt, tw, th, lds2, 2}, r);
            }
        }
    }
    const int c = m < cap ? m : cap;
    for (int i = 0; i < c; ++i) out[i] = all[i];
    return c;
}

// Picks the scale count and tile of the stage starting at scale j0 (at most
// `left` scales remain): the largest ns <= 3 that has a tile, with its best
// tile.  Returns false if no tile exists even for one scale.
template <typename T>
static bool pick_stage(int n, int j0, int left, bool noise, StageGeom* g) {
    for (int ns = left < 3 ? left : 3; ns >= 1; --ns)
        if (stage_candidates<T>(n, j0, ns, noise, g, 1) == 1) return true;
    return false;
}

// The geometry of a given tile (as the planner would size it).
template <typename T>
static bool stage_geom_of(int n, int j0, int ns, int tw, int th, int rb, bool noise,
                          StageGeom* g) {
    StageGeom all[kMaxCand];
    const int m = stage_candidates<T>(n, j0, ns, noise, all, kMaxCand);
    for (int i = 0; i < m; ++i)
        if (all[i].tw == tw && all[i].th == th && all[i].rb == rb) {
            *g = all[i];
            return true;
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

template <typename T, int NT, int NS, int KV, int RB>
static hipError_t launch_noise_stage_nt(const NoiseStageArgs<T>& a, const StageGeom& g, int tiles,
                                        hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_starlet_noise_stage<T, NT, NS, KV, RB, false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_starlet_noise_stage<T, NT, NS, KV, RB, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (a.img_logd < 0 || a.img_logd >= a.j0 || a.cout_logd < 0 || a.cout_logd >= a.logn - a.img_logd)
        return hipErrorInvalidValue;
    {  // the tile must fit the prefetch registers and the owned vectors of the threads
        constexpr int G = Vec<T>::G;
        const int d0 = 1 << (a.j0 - 1 - a.img_logd);
        const int TXT = g.tw + 2 * stage_hx(d0, NS, G), TVT = g.th + 2 * 2 * ((1 << NS) - 1);
        if ((TXT / G) * TVT > NT * noise_prefetch(NT, KV, RB) || g.tw * g.th > NT * KV * G ||
            !grid_fits(TXT, G, NT, NS) ||
            g.lds < (size_t)(2 * RB * (TXT + 2 * G) * TVT + G) * sizeof(T))
            return hipErrorInvalidConfiguration;
    }
    static const char* names[12] = {"noise_stage_j1", "noise_stage_j2", "noise_stage_j3",
                                    "noise_stage_j4", "noise_stage_j5", "noise_stage_j6",
                                    "noise_stage_j7", "noise_stage_j8", "noise_stage_j9",
                                    "noise_stage_j10", "noise_stage_j11", "noise_stage_j12"};
    if (a.cout_logd > 0)
        AMAP_LAUNCH(names[a.j0 - 1 < 12 ? a.j0 - 1 : 11], s,
                    k_starlet_noise_stage<T, NT, NS, KV, RB, true><<<dim3(tiles, a.groups), NT, g.lds, s>>>(a));
    else
        AMAP_LAUNCH(names[a.j0 - 1 < 12 ? a.j0 - 1 : 11], s,
                    k_starlet_noise_stage<T, NT, NS, KV, RB, false><<<dim3(tiles, a.groups), NT, g.lds, s>>>(a));
    return hipGetLastError();
}

template <typename T, int NS>
static hipError_t launch_noise_stage_ns(const NoiseStageArgs<T>& a, const StageGeom& g, int tiles,
                                        hipStream_t s) {
    const NoiseCfg cfg = noise_cfg(g.tw * g.th / Vec<T>::G);
    if (cfg.kv == 4) {
        if constexpr (NS < 3) {
            if (g.rb == 1) return launch_noise_stage_nt<T, 512, NS, 4, 1>(a, g, tiles, s);
        }
        return hipErrorInvalidConfiguration;
    }
    if (g.rb == 2) {  // float stages of one or two scales only
        if constexpr (sizeof(T) == 4 && NS < 3) {
            switch (cfg.nt) {
                case 256: return launch_noise_stage_nt<T, 256, NS, 1, 2>(a, g, tiles, s);
                case 512: return launch_noise_stage_nt<T, 512, NS, 1, 2>(a, g, tiles, s);
                case 1024: return launch_noise_stage_nt<T, 1024, NS, 1, 2>(a, g, tiles, s);
                default: return hipErrorInvalidValue;
            }
        }
        return hipErrorInvalidConfiguration;
    }
    if (g.rb != 1) return hipErrorInvalidValue;
    switch (cfg.nt) {
        case 256: return launch_noise_stage_nt<T, 256, NS, 1, 1>(a, g, tiles, s);
        case 512: return launch_noise_stage_nt<T, 512, NS, 1, 1>(a, g, tiles, s);
        case 1024:  // double-precision tiles of 1024 vectors run 512 threads x 4 instead
            if constexpr (sizeof(T) == 4) return launch_noise_stage_nt<T, 1024, NS, 1, 1>(a, g, tiles, s);
            return hipErrorInvalidConfiguration;
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_noise_stage(const NoiseStageArgs<T>& a, const StageGeom& g, int tiles,
                                     hipStream_t s) {
    switch (a.ns) {
        case 1: return launch_noise_stage_ns<T, 1>(a, g, tiles, s);
        case 2: return launch_noise_stage_ns<T, 2>(a, g, tiles, s);
        case 3: return launch_noise_stage_ns<T, 3>(a, g, tiles, s);
        default: return hipErrorInvalidValue;
    }
}

// Final noise stages on whole sub-grids: side m = n / d0 from 16 to 64
// (float; 32 for double, whose vectors hold two values), at most four scales
// (three for double, so that the partials of several groups stay within
// starlet_partials_bytes).
template <typename T>
static bool subgrid_ok(int n, int j0, int J) {
    const int ns = J - j0;
    if (j0 < 1 || ns < 1 || ns > (sizeof(T) == 4 ? 4 : 3)) return false;
    const int d0 = 1 << (j0 - 1);
    if (d0 > n / 16) return false;
    const int m = n / d0;
    return m >= 16 && m <= (sizeof(T) == 4 ? 64 : 32);
}

// A noise tile stage on the sub-grids of d0 = 2^(j0-1) as periodic images
// of side m = n / d0: the geometry of the tile (tw, th, rb) of an m x m
// map's first stage of ns scales.  False if the planner offers no such tile.
template <typename T>
static bool images_geom(int n, int j0, int ns, int tw, int th, int rb, StageGeom* g) {
    if (j0 < 2 || ns < 1 || ns > 3 || (n >> (j0 - 1)) < 16) return false;
    return stage_geom_of<T>(n >> (j0 - 1), 1, ns, tw, th, rb, true, g);
}

// LDS of a sub-grid stage: RB tiles of m rows of m values, twice.
template <typename T>
constexpr size_t subgrid_lds_bytes(int logm, int rb) {
    return 2 * (size_t)rb * (1 << logm) * (1 << logm) * sizeof(T);
}

template <typename T, int LOGM, int NS>
static hipError_t launch_subgrid_nsm(const NoiseSubArgs<T>& a, int tiles, hipStream_t s) {
    constexpr int NT = (1 << (2 * LOGM)) / Vec<T>::G;
    if (a.rb != 1 && a.rb != 2) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_starlet_noise_subgrid<T, LOGM, NS, 1>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_starlet_noise_subgrid<T, LOGM, NS, 2>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const size_t lds = subgrid_lds_bytes<T>(LOGM, a.rb);
    if (lds > (size_t)kLdsBytes) return hipErrorInvalidConfiguration;
    static const char* names[12] = {"noise_stage_j1", "noise_stage_j2", "noise_stage_j3",
                                    "noise_stage_j4", "noise_stage_j5", "noise_stage_j6",
                                    "noise_stage_j7", "noise_stage_j8", "noise_stage_j9",
                                    "noise_stage_j10", "noise_stage_j11", "noise_stage_j12"};
    if (a.rb == 2)
        AMAP_LAUNCH(names[a.j0 - 1 < 12 ? a.j0 - 1 : 11], s,
                    k_starlet_noise_subgrid<T, LOGM, NS, 2><<<dim3(tiles, a.groups), NT, lds, s>>>(a));
    else
        AMAP_LAUNCH(names[a.j0 - 1 < 12 ? a.j0 - 1 : 11], s,
                    k_starlet_noise_subgrid<T, LOGM, NS, 1><<<dim3(tiles, a.groups), NT, lds, s>>>(a));
    return hipGetLastError();
}

template <typename T, int LOGM>
static hipError_t launch_subgrid_m(const NoiseSubArgs<T>& a, int ns, int tiles, hipStream_t s) {
    switch (ns) {
        case 1: return launch_subgrid_nsm<T, LOGM, 1>(a, tiles, s);
        case 2: return launch_subgrid_nsm<T, LOGM, 2>(a, tiles, s);
        case 3: return launch_subgrid_nsm<T, LOGM, 3>(a, tiles, s);
        case 4:
            if constexpr (sizeof(T) == 4) return launch_subgrid_nsm<T, LOGM, 4>(a, tiles, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_subgrid(const NoiseSubArgs<T>& a, int ns, int logm, int tiles, hipStream_t s) {
    switch (logm) {
        case 4: return launch_subgrid_m<T, 4>(a, ns, tiles, s);
        case 5: return launch_subgrid_m<T, 5>(a, ns, tiles, s);
        case 6:
            if constexpr (sizeof(T) == 4) return launch_subgrid_m<T, 6>(a, ns, tiles, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

// Workgroups of a noise stage: one per tile, times enough realisation groups
// to give every CU work (256 of them), at most one group per realisation.
static int noise_groups(int tiles, int batch) {
    int g = 256 / tiles;
    if (g < 1) g = 1;
    if (g > batch) g = batch;
    return g;
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
bool starlet_all_tiled(int n, int J) {
    for (int j0 = 1; j0 < J;) {
        StageGeom g{};
        if (!pick_stage<T>(n, j0, J - j0, false, &g)) return false;
        j0 += g.ns;
    }
    return true;
}
// The analytic planner's noise stages up to the first scale from which a
// sub-grid final stage applies, then that stage.  False if there is no such
// scale or a stage before it has no LDS tile.
template <typename T>
bool analytic_subgrid_plan(int n, int J, StagePlan* out) {
    out->nstages = 0;
    int js = 0;  // the first scale a sub-grid stage can start at
    for (int j = 1; j < J && !js; ++j)
        if (subgrid_ok<T>(n, j, J)) js = j;
    if (!js) return false;
    for (int j0 = 1; j0 < js;) {
        StageGeom g{};
        if (!pick_stage<T>(n, j0, js - j0, true, &g) || out->nstages >= 15) {
            out->nstages = 0;
            return false;
        }
        out->st[out->nstages++] = StagePlan::Stage{j0, g.ns, g.tw, g.th, g.rb, 0};
        j0 += g.ns;
    }
    out->st[out->nstages++] = StagePlan::Stage{js, J - js, n >> (js - 1), n >> (js - 1), 2, 1};
    return true;
}
template bool analytic_subgrid_plan<float>(int, int, StagePlan*);
template bool analytic_subgrid_plan<double>(int, int, StagePlan*);

// True if plan is a schedule launch_starlet accepts for an n x n, J-plane
// transform (noise statistics or plane output): consecutive stages from
// scale 1 to J-1, each with a tile the planner offers for its start and
// scale count (or, last and for noise only, a valid sub-grid stage).
template <typename T>
bool plan_valid(int n, int J, bool noise, const StagePlan& plan) {
    if (plan.nstages < 1 || plan.nstages > 16) return false;
    int j = 1;
    for (int k = 0; k < plan.nstages; ++k) {
        const StagePlan::Stage& t = plan.st[k];
        if (t.j0 != j || t.ns < 1 || t.j0 + t.ns > J) return false;
        if (t.kind == kStageSubgrid) {
            if (!noise || k + 1 != plan.nstages || t.j0 + t.ns != J || !subgrid_ok<T>(n, t.j0, J) ||
                (t.rb != 1 && t.rb != 2) || t.tw != (n >> (t.j0 - 1)) || t.th != t.tw)
                return false;
        } else if (t.kind == kStageImages) {
            // after a plain tile stage or another such stage; the last stage or
            // followed by another such stage or the final sub-grid stage
            StageGeom g{};
            if (!noise || k == 0 || plan.st[k - 1].kind == kStageSubgrid ||
                (k + 1 < plan.nstages && plan.st[k + 1].kind == kStageTile) || t.ns > 3 ||
                !images_geom<T>(n, t.j0, t.ns, t.tw, t.th, t.rb, &g))
                return false;
        } else if (t.kind == kStageTile) {
            StageGeom g{};
            if (t.ns > 3 || !stage_geom_of<T>(n, t.j0, t.ns, t.tw, t.th, t.rb, noise, &g)) return false;
        } else {
            return false;
        }
        j += t.ns;
    }
    return j == J;
}
template bool plan_valid<float>(int, int, bool, const StagePlan&);
template bool plan_valid<double>(int, int, bool, const StagePlan&);

template bool starlet_all_tiled<float>(int, int);
template bool starlet_all_tiled<double>(int, int);

template <typename T>
hipError_t launch_starlet(const StarletArgs<T>& a) {
    const int n = 1 << a.logn;
    const long long n2 = (long long)n * n;
    const bool acc = a.M != nullptr;
    // plan the stages: (j0, ns, tile) or a per-scale stage (tile.nt == 0)
    struct Stage { int j0, ns; StageGeom g; bool tiled, sub, images; };
    Stage plan[16];
    int nstages = 0;
    if (a.plan && a.plan->nstages > 0) {
        // a tuned schedule (possibly a single stage, for timing it)
        for (int k = 0; k < a.plan->nstages; ++k) {
            const StagePlan::Stage& t = a.plan->st[k];
            StageGeom g{};
            if (t.kind == kStageSubgrid) {  // a final noise stage on whole sub-grids
                if (!acc || k + 1 != a.plan->nstages || t.j0 + t.ns != a.J || !subgrid_ok<T>(n, t.j0, a.J) ||
                    (t.rb != 1 && t.rb != 2))
                    return hipErrorInvalidValue;
                g.rb = t.rb;
                plan[nstages++] = Stage{t.j0, t.ns, g, false, true, false};
                continue;
            }
            if (t.kind == kStageImages) {  // noise tiles on sub-grid images
                if (!acc || (k > 0 && a.plan->st[k - 1].kind == kStageSubgrid) ||
                    (k + 1 < a.plan->nstages && a.plan->st[k + 1].kind == kStageTile) ||
                    !images_geom<T>(n, t.j0, t.ns, t.tw, t.th, t.rb, &g))
                    return hipErrorInvalidValue;
                plan[nstages++] = Stage{t.j0, t.ns, g, true, false, true};
                continue;
            }
            if (t.kind != kStageTile || !stage_geom_of<T>(n, t.j0, t.ns, t.tw, t.th, t.rb, acc, &g))
                return hipErrorInvalidValue;
            plan[nstages++] = Stage{t.j0, t.ns, g, true, false, false};
        }
    } else {
        for (int j0 = 1; j0 < a.J; ) {
            StageGeom g{};
            const bool tiled = pick_stage<T>(n, j0, a.J - j0, acc, &g);
            const int ns = tiled ? g.ns : 1;
            plan[nstages++] = Stage{j0, ns, g, tiled, false, false};
            j0 += ns;
        }
    }
    if (a.planes_off) {
        // grouped maps: c ping-pongs between cbuf0 and cbuf1; the last stage
        // writes c_{J-1} into each map's last plane
        if (acc || !a.cbuf0 || !a.cbuf1) return hipErrorInvalidValue;
        const T* cur = a.kappa_off ? nullptr : a.kappa;  // keeps the first stage's output off its input
        for (int gi = 0; gi < nstages; ++gi) {
            const Stage& st = plan[gi];
            if (!st.tiled) return hipErrorNotSupported;
            const bool last = st.j0 + st.ns == a.J;
            int lt = 0;
            while ((1 << lt) < st.g.tw) ++lt;
            StageArgs<T> s;
            s.logn = a.logn; s.j0 = st.j0; s.ns = st.ns; s.log_tw = lt; s.th = st.g.th;
            s.src = gi == 0 ? a.kappa : cur; s.src_stride = n2; s.src_off = gi == 0 ? a.kappa_off : nullptr;
            s.planes = a.planes; s.planes_stride = 0; s.planes_off = a.planes_off; s.plane_base = 0;
            T* dst = last ? nullptr : (cur == a.cbuf0 ? a.cbuf1 : a.cbuf0);
            s.cout = dst; s.cout_stride = n2; s.cout_plane = last ? a.J - 1 : -1;
            const hipError_t e = launch_stage<T>(s, st.g, a.batch, a.stream);
            if (e != hipSuccess) return e;
            cur = dst;
        }
        return hipGetLastError();
    }
    T* final_c = acc ? nullptr : a.planes + (long long)(a.J - 1) * n2;
    const long long final_stride = a.planes_stride;
    const T* cur = a.kappa;
    long long cur_stride = a.in_stride;
    if (acc && a.in_stride != n2) return hipErrorInvalidValue;  // realisations are packed
    for (int gi = 0; gi < nstages; ++gi) {
        const Stage& st = plan[gi];
        const bool last = st.j0 + st.ns == a.J;
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
        int lt = 0;
        while ((1 << lt) < st.g.tw) ++lt;
        if (st.sub) {  // acc only, the last stage: c and the statistics in sub-grid order
            // (after a stage on sub-grid images, their sub-grids image by image)
            const int d0 = 1 << (st.j0 - 1);
            const int tiles = d0 * d0;
            int logm = 0;
            while ((1 << logm) < n / d0) ++logm;
            NoiseSubArgs<T> s;
            s.logn = a.logn; s.j0 = st.j0; s.src = cur; s.batch = a.batch; s.rb = st.g.rb;
            s.groups = noise_groups(tiles, a.batch); s.done = a.done;
            s.M = a.M + (long long)(st.j0 - 1) * n2; s.M2 = a.M2 + (long long)(st.j0 - 1) * n2;
            s.part = a.part;
            {
                using AccT = typename std::conditional<sizeof(T) == 8, double, float>::type;
                if (s.groups > 1 && (size_t)s.groups * st.ns * 2 * (size_t)n2 * sizeof(AccT) >
                                        starlet_partials_bytes(a.logn, a.batch))
                    return hipErrorInvalidConfiguration;
            }
            e = launch_subgrid<T>(s, st.ns, logm, tiles, a.stream);
            if (e == hipSuccess && s.groups > 1) {
                using AccT = typename std::conditional<sizeof(T) == 8, double, float>::type;
                AMAP_LAUNCH("merge_partials", a.stream,
                            k_merge_partials<AccT><<<(unsigned)((n2 + 255) / 256), 256, 0, a.stream>>>(
                                static_cast<const AccT*>(a.part), s.groups, st.ns, a.batch, a.done,
                                n2, s.M, s.M2));
                e = hipGetLastError();
            }
            if (e != hipSuccess) return e;
            continue;
        }
        if (st.tiled && acc) {
            // on sub-grid images (of side nm), the stage starts at dilation 1 there
            const int li = st.images ? st.j0 - 1 : 0;
            const int d0 = 1 << (st.j0 - 1 - li), nm = n >> li;
            const int tiles = ((nm / st.g.tw) * ((nm / d0) / st.g.th) * d0) << (2 * li);
            NoiseStageArgs<T> s;
            s.logn = a.logn; s.j0 = st.j0; s.ns = st.ns; s.log_tw = lt; s.th = st.g.th;
            s.src = cur; s.cout = dst; s.batch = a.batch;
            s.groups = noise_groups(tiles, a.batch); s.done = a.done;
            s.M = a.M + (long long)(st.j0 - 1) * n2; s.M2 = a.M2 + (long long)(st.j0 - 1) * n2;
            s.part = a.part;
            s.inv_tvec = 1.0f / (float)((st.g.tw + 2 * stage_hx(d0, st.ns, Vec<T>::G)) / Vec<T>::G);
            // a following sub-grid or sub-grid image stage reads c in its
            // sub-grid order (within each image of this one)
            s.img_logd = li;
            s.cout_logd = (gi + 1 < nstages && (plan[gi + 1].sub || plan[gi + 1].images))
                              ? plan[gi + 1].j0 - 1 - li
                              : (a.plan && nstages == 1 && dst ? a.plan->cout_logd : 0);
            {
                using AccT = typename std::conditional<sizeof(T) == 8, double, float>::type;
                if (s.groups > 1 && (size_t)s.groups * st.ns * 2 * (size_t)n2 * sizeof(AccT) >
                                        starlet_partials_bytes(a.logn, a.batch))
                    return hipErrorInvalidConfiguration;
            }
            e = launch_noise_stage<T>(s, st.g, tiles, a.stream);
            if (e == hipSuccess && s.groups > 1) {
                using AccT = typename std::conditional<sizeof(T) == 8, double, float>::type;
                AMAP_LAUNCH("merge_partials", a.stream,
                            k_merge_partials<AccT><<<(unsigned)((n2 + 255) / 256), 256, 0, a.stream>>>(
                                static_cast<const AccT*>(a.part), s.groups, st.ns, a.batch, a.done,
                                n2, s.M, s.M2));
                e = hipGetLastError();
            }
            if (e != hipSuccess) return e;
            cur = dst;
            cur_stride = dst_stride;
            continue;
        }
        if (st.tiled) {
            StageArgs<T> s;
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

// Groups x scales x (mean, M2) x pixels in the accumulator type, bounded by
// 256 groups of the largest tile (4096 pixels) and by one group per
// realisation.
// Partials of a multi-group noise stage: groups x ns x 2 planes of the
// accumulator type, groups <= min(batch, 256 / tiles).  Three-scale stages
// use tiles of at most 4096 pixels, so groups x n^2 <= 256 x 4096 and the
// bound below is 3 x 2 x 8 bytes per such pixel; two-scale float stages may
// use 8192-pixel tiles, needing 2 x 2 x 4 bytes per pixel of 256 x 8192,
// which is less.  launch_starlet checks each stage against it.
size_t starlet_partials_bytes(int logn, int batch) {
    const long long n2 = 1ll << (2 * logn);
    long long px = 256ll * 4096;
    if ((long long)batch * n2 < px) px = (long long)batch * n2;
    return (size_t)(3 * 2 * px) * sizeof(double);
}

template <typename T>
hipError_t launch_reconstruct(int logn, int J, const T* planes, T* out, hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    AMAP_LAUNCH("reconstruct", s,
                k_reconstruct<T><<<(unsigned)((n2 + 255) / 256), 256, 0, s>>>(planes, out, logn, J));
    return hipGetLastError();
}

// AMAP_TUNE_LOG=1 in the environment prints every timed candidate.
static bool tune_log() {
    static const bool on = [] {
        const char* v = std::getenv("AMAP_TUNE_LOG");
        return v && v[0] && v[0] != '0';
    }();
    return on;
}

template <typename T>
hipError_t tune_starlet(const StarletArgs<T>& a, int reps, StagePlan* out) {
    const int n = 1 << a.logn, J = a.J;
    const bool acc = a.M != nullptr;
    if (J < 2 || J > 16 || reps < 1) return hipErrorInvalidValue;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(a.stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return hipErrorNotSupported;  // timing needs a live stream
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // the average time of one stage alone (reps launches after a warm one)
    auto time_stage = [&](const StagePlan::Stage& st, float* us, int cout_logd = 0) {
        StagePlan sub;
        sub.nstages = 1;
        sub.st[0] = st;
        sub.cout_logd = cout_logd;
        StarletArgs<T> b = a;
        b.plan = &sub;
        if (st.j0 > 1 && b.planes_off) {  // grouped: later stages read the c buffers
            b.kappa = b.cbuf0;
            b.kappa_off = nullptr;
        }
        hipError_t r = launch_starlet<T>(b);  // warm
        if (r == hipSuccess) r = hipEventRecord(e0, a.stream);
        for (int k = 0; k < reps && r == hipSuccess; ++k) r = launch_starlet<T>(b);
        if (r == hipSuccess) r = hipEventRecord(e1, a.stream);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        float ms = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        *us = 1e3f * ms / reps;
        if (r == hipSuccess && tune_log()) {
            const char* kind = st.kind == kStageSubgrid ? "sub-grids" : st.kind == kStageImages ? "image tile" : "tile";
            std::fprintf(stderr, "amap tune: n=%d J=%d %s batch=%d stage j0=%d ns=%d %s %dx%d rb=%d: %.1f us\n",
                         n, J, acc ? "noise" : "signal", a.batch, st.j0, st.ns, kind, st.tw, st.th, st.rb, *us);
        }
        return r;
    };
    // the two best tiles (least halo overhead) of each thread configuration
    // (threads, owned vectors, realisations per pass) of a stage of ns
    // scales from j0 of an m x m map
    auto candidates = [&](int m, int j0, int ns, StageGeom* cand) {
        StageGeom all[kMaxCand];
        const int na = stage_candidates<T>(m, j0, ns, acc, all, kMaxCand);
        auto config = [&](const StageGeom& sg) {
            const NoiseCfg cfg = noise_cfg(sg.tw * sg.th / Vec<T>::G);
            return acc ? (cfg.nt * 8 + cfg.kv) * 4 + sg.rb : sg.nt;
        };
        int nc = 0;
        for (int i = 0; i < na && nc < 24; ++i) {
            const int key = config(all[i]);
            int same = 0;
            for (int q = 0; q < nc; ++q) same += config(cand[q]) == key;
            if (same < 2) cand[nc++] = all[i];
        }
        return nc;
    };
    // best[j]: least time for scales j .. J-1 from c_{j-1} in natural order,
    // pick[j] its first stage, then_images[j] whether a stage on sub-grid
    // images follows it; img[j]: least time for scales j .. J-1 starting with
    // a stage on sub-grid images, img_pick[j] that stage and img_next[j] what
    // follows it (0 nothing, 1 the final sub-grid stage, 2 another stage on
    // sub-grid images); sub[j]: the final sub-grid stage from j, sub_pick[j] it.
    float best[18], img[18], sub[18];
    StagePlan::Stage pick[18], img_pick[18], sub_pick[18];
    bool then_images[18];
    int img_next[18];
    best[J] = 0.f;
    img[J] = sub[J] = -1.f;
    for (int j = J - 1; j >= 1 && e == hipSuccess; --j) {
        best[j] = img[j] = sub[j] = -1.f;
        then_images[j] = false;
        img_next[j] = 0;
        for (int rb = 1; rb <= 2 && acc && e == hipSuccess && subgrid_ok<T>(n, j, J); ++rb) {
            // all remaining scales on whole sub-grids (a final stage)
            const int m = n >> (j - 1);
            const StagePlan::Stage st{j, J - j, m, m, rb, kStageSubgrid};
            float t = 0.f;
            e = time_stage(st, &t);
            if (e == hipSuccess && (sub[j] < 0.f || t < sub[j])) {
                sub[j] = t;
                sub_pick[j] = st;
            }
        }
        // a tile stage on the sub-grid images of d0 = 2^(j-1)
        for (int ns = 1; ns <= 3 && acc && j >= 2 && j + ns <= J && (n >> (j - 1)) >= 16 && e == hipSuccess; ++ns) {
            // what follows: nothing, the final sub-grid stage or another images stage
            float tail = j + ns == J ? 0.f : -1.f;
            int next = 0;
            if (j + ns < J) {
                if (sub[j + ns] >= 0.f) { tail = sub[j + ns]; next = 1; }
                if (img[j + ns] >= 0.f && (tail < 0.f || img[j + ns] < tail)) { tail = img[j + ns]; next = 2; }
            }
            if (tail < 0.f) continue;
            StageGeom cand[24];
            const int nc = candidates(n >> (j - 1), 1, ns, cand);
            for (int c = 0; c < nc && e == hipSuccess; ++c) {
                const StagePlan::Stage st{j, ns, cand[c].tw, cand[c].th, cand[c].rb, kStageImages};
                float t = 0.f;
                e = time_stage(st, &t, next ? ns : 0);  // the next stage's d over this one's
                if (e == hipSuccess && (img[j] < 0.f || t + tail < img[j])) {
                    img[j] = t + tail;
                    img_pick[j] = st;
                    img_next[j] = next;
                }
            }
        }
        for (int ns = 1; ns <= 3 && j + ns <= J && e == hipSuccess; ++ns) {
            const float rest = best[j + ns], rest_img = img[j + ns];
            if (rest < 0.f && rest_img < 0.f) continue;
            const bool via_img = rest_img >= 0.f && (rest < 0.f || rest_img < rest);
            // before a stage on sub-grids the coarse output goes out in their order
            const bool to_sub = via_img || (j + ns < J && pick[j + ns].kind == kStageSubgrid);
            StageGeom cand[24];
            const int nc = candidates(n, j, ns, cand);
            for (int c = 0; c < nc && e == hipSuccess; ++c) {
                const StagePlan::Stage st{j, ns, cand[c].tw, cand[c].th, cand[c].rb, kStageTile};
                float t = 0.f;
                e = time_stage(st, &t, acc && to_sub ? j + ns - 1 : 0);
                const float total = t + (via_img ? rest_img : rest);
                if (e == hipSuccess && (best[j] < 0.f || total < best[j])) {
                    best[j] = total;
                    pick[j] = st;
                    then_images[j] = via_img;
                }
            }
        }
        if (sub[j] >= 0.f && (best[j] < 0.f || sub[j] < best[j])) {
            best[j] = sub[j];
            pick[j] = sub_pick[j];
            then_images[j] = false;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    if (best[1] < 0.f) return hipErrorNotSupported;  // some stage start has no tile
    out->nstages = 0;
    for (int j = 1; j < J;) {
        const bool to_img = then_images[j];
        out->st[out->nstages++] = pick[j];
        j += pick[j].ns;
        while (to_img && j < J) {  // the chain of stages on sub-grid images
            const int next = img_next[j];
            out->st[out->nstages++] = img_pick[j];
            j += img_pick[j].ns;
            if (next == 1) out->st[out->nstages++] = sub_pick[j];
            if (next != 2) j = J;
        }
    }
    return hipSuccess;
}
template hipError_t tune_starlet<float>(const StarletArgs<float>&, int, StagePlan*);
template hipError_t tune_starlet<double>(const StarletArgs<double>&, int, StagePlan*);

template hipError_t launch_starlet<float>(const StarletArgs<float>&);
template hipError_t launch_starlet<double>(const StarletArgs<double>&);
template hipError_t launch_reconstruct<float>(int, int, const float*, float*, hipStream_t);
template hipError_t launch_reconstruct<double>(int, int, const double*, double*, hipStream_t);

}  // namespace amap

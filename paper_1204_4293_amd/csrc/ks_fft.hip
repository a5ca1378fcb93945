// Kaiser-Squires inversion on the GPU: a two-dimensional complex FFT with the
// spectral multiply by conj(D(k)) fused between the forward and inverse
// transforms along x.
//
// Pass structure for one n x n map (columns first, so that the row pass sees
// whole spectral rows and can apply the KS kernel between its forward and
// inverse transforms):
//   P1  column strips:  (g1 + i g2) [optionally rotated by Philox phases]
//                       -> forward FFT along y             -> C
//   P2  whole rows:     forward FFT along x, multiply by conj(D)/n^2,
//                       inverse FFT along x                -> C
//   P3  column strips:  inverse FFT along y -> kappa_E = Re, kappa_B = Im
// A strip is W adjacent columns, so every HBM access is a W-element row
// segment; a row pass reads and writes whole rows.
//
// Each length-N transform is a four-step FFT with N = N1 * N2: every thread
// holds N1 (then N2) values in registers and runs a radix-2 DFT on them with
// compile-time twiddles, the inter-step twiddles come from a table, and one
// LDS exchange separates the two steps.  Along x a transform's N2 threads
// sit in one wavefront, so the exchange needs no workgroup barrier, and the
// inverse transform starts from the forward output exactly as each thread
// holds it.  Float64 from 1024 points, whose per-thread DFTs would not fit
// the register file, uses radix-4 Stockham passes held in LDS instead.
#include "amap_device.h"
#include "amap_launch.h"
#include "fft_reg.h"

namespace amap {

// K consecutive values at p (16-byte aligned) through 16-byte loads.
template <typename T, int K>
__device__ __forceinline__ void load16(const T* __restrict__ p, T (&out)[K]) {
    if constexpr (sizeof(T) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int i = 0; i < K / 4; ++i) {
            const f4 v = reinterpret_cast<const f4*>(p)[i];
            out[4 * i] = v[0]; out[4 * i + 1] = v[1]; out[4 * i + 2] = v[2]; out[4 * i + 3] = v[3];
        }
    } else {
        typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int i = 0; i < K / 2; ++i) {
            const d2 v = reinterpret_cast<const d2*>(p)[i];
            out[2 * i] = v[0]; out[2 * i + 1] = v[1];
        }
    }
}

// ---- in-LDS Stockham FFT ---------------------------------------------------
// Element (line l, index i) of LINES interleaved lines of length 2^LOGN
// lives at buf[i*IS + l*LS].  NT threads cooperate.  Each stage reads all of
// a thread's butterfly inputs into registers, synchronises, and writes the
// outputs in place at their Stockham positions, so one buffer suffices.
// LINES_FAST picks which index consecutive threads walk (the one with unit
// stride in LDS, to keep the banks conflict-free on reads).
template <typename T, int LOGN, int LINES, int NT, int IS, int LS, bool LINES_FAST, bool INV>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, const cpx<T>* __restrict__ tw) {
    constexpr int N = 1 << LOGN;
    const int tid = threadIdx.x;
    int Ls = 1;
#pragma unroll
    for (int st = 0; st < LOGN / 2; ++st) {
        constexpr int NB = (N / 4) * LINES;
        constexpr int PER = (NB + NT - 1) / NT;
        cpx<T> v[PER][4];
        int base[PER], lo[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int t = tid + q * NT;
            if (NB % NT == 0 || t < NB) {
                int l, j;
                if (LINES_FAST) { l = t % LINES; j = t / LINES; }
                else            { j = t % (N / 4); l = t / (N / 4); }
                const int k = j & (Ls - 1);
                cpx<T> a[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) a[p] = buf[(j + p * (N / 4)) * IS + l * LS];
                if (st > 0) {
                    const int unit = kMaxN / (4 * Ls);
#pragma unroll
                    for (int p = 1; p < 4; ++p) {
                        const cpx<T> w = tw[p * k * unit];
                        a[p] = INV ? cmulc(a[p], w) : cmul(a[p], w);
                    }
                }
                const cpx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
                const cpx<T> t2 = a[1] + a[3], t3 = rot90<T, INV>(a[1] - a[3]);
                v[q][0] = t0 + t2;
                v[q][1] = t1 + t3;
                v[q][2] = t0 - t2;
                v[q][3] = t1 - t3;
                base[q] = (j - k) * 4 + k;
                lo[q] = l * LS;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int t = tid + q * NT;
            if (NB % NT == 0 || t < NB) {
#pragma unroll
                for (int p = 0; p < 4; ++p) buf[(base[q] + p * Ls) * IS + lo[q]] = v[q][p];
            }
        }
        __syncthreads();
        Ls *= 4;
    }
    if (LOGN & 1) {
        constexpr int NB = (N / 2) * LINES;
        constexpr int PER = (NB + NT - 1) / NT;
        cpx<T> v[PER][2];
        int base[PER], lo[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int t = tid + q * NT;
            if (NB % NT == 0 || t < NB) {
                int l, j;
                if (LINES_FAST) { l = t % LINES; j = t / LINES; }
                else            { j = t % (N / 2); l = t / (N / 2); }
                const int k = j & (Ls - 1);
                cpx<T> a0 = buf[j * IS + l * LS];
                cpx<T> a1 = buf[(j + N / 2) * IS + l * LS];
                if (Ls > 1) {
                    const cpx<T> w = tw[k * (kMaxN / (2 * Ls))];
                    a1 = INV ? cmulc(a1, w) : cmul(a1, w);
                }
                v[q][0] = a0 + a1;
                v[q][1] = a0 - a1;
                base[q] = (j - k) * 2 + k;
                lo[q] = l * LS;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int t = tid + q * NT;
            if (NB % NT == 0 || t < NB) {
                buf[base[q] * IS + lo[q]] = v[q][0];
                buf[(base[q] + Ls) * IS + lo[q]] = v[q][1];
            }
        }
        __syncthreads();
    }
}

// ---- launch geometry ---------------------------------------------------------
// Column strips: W columns x full height in LDS, at most 128 KiB.
template <typename T, int LOGN>
struct StripCfg {
    static constexpr int N = 1 << LOGN;
    static constexpr int LDS_ELEMS = (128 * 1024) / (int)sizeof(cpx<T>);
    static constexpr int W0 = LDS_ELEMS / N;
    static constexpr int W = W0 > 16 ? 16 : W0;
    static constexpr int NT0 = (N / 4) * W;
    static constexpr int NT = NT0 > 512 ? 512 : (NT0 < 64 ? 64 : NT0);
};
// Whole rows: ROWS rows per workgroup of NT threads.
template <typename T, int LOGN>
struct RowCfg {
    static constexpr int N = 1 << LOGN;
    static constexpr int NT = 256;
    static constexpr int ROWS0 = (4 * NT / N) > 1 ? (4 * NT / N) : 1;
    static constexpr int ROWS = ROWS0 > N ? N : ROWS0;
};

__device__ __forceinline__ int signed_freq(int i, int n) { return i < n / 2 ? i : i - n; }

// Reciprocal: the hardware estimate (1 ulp) in single precision, a rounded
// division in double.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// ---- P1: load shears (optionally rotate), forward FFT along y -------------------
// grid: (n / W strips, batch).  Map b reads g1 + b*g_stride (g_stride = 0 when
// every batch entry is a noise realisation of the same map) and writes
// C + b*n*n.  Realisation index r = r0 + b.
template <typename T, int LOGN, bool ROTATE>
__global__ void __launch_bounds__((StripCfg<T, LOGN>::NT))
k_ks_cols_fwd_generic(const T* __restrict__ g1, const T* __restrict__ g2, long long g_stride,
              const long long* __restrict__ g1_off, const long long* __restrict__ g2_off,
              cpx<T>* __restrict__ C, uint64_t seed, uint64_t r0,
              const cpx<T>* __restrict__ tw) {
    using Cfg = StripCfg<T, LOGN>;
    constexpr int N = Cfg::N, W = Cfg::W, NT = Cfg::NT;
    __shared__ cpx<T> buf[N * W];
    const int b = blockIdx.y;
    const int x0 = blockIdx.x * W;
    const T* a1 = g1 + (g1_off ? g1_off[b] : (long long)b * g_stride);
    const T* a2 = g2 + (g2_off ? g2_off[b] : (long long)b * g_stride);
    if (ROTATE) {
        // one Philox block covers 8 consecutive pixels of a row
        constexpr int OCT_PER_ROW = (W + 7) / 8;
        const uint64_t r = r0 + b;
        for (int o = threadIdx.x; o < N * OCT_PER_ROW; o += NT) {
            const int y = o / OCT_PER_ROW;
            const int cx = (o % OCT_PER_ROW) * 8;                // column offset in strip
            const int xa = (W >= 8) ? (x0 + cx) : (x0 & ~7);      // first pixel of the octet
            const uint64_t pix = (uint64_t)y * N + xa;
            uint32_t u[8];
            philox_block_u32(seed, r, pix >> 3, u);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int x = xa + i;
                if (W < 8 && (x < x0 || x >= x0 + W)) continue;
                T p = a1[(long long)y * N + x], q = a2[(long long)y * N + x];
                rotate_by_u32(u[i], p, q);
                buf[y * W + (x - x0)] = make_cpx(p, q);
            }
        }
    } else {
        for (int e = threadIdx.x; e < N * W; e += NT) {
            const int y = e / W, c = e % W;
            const long long gi = (long long)y * N + x0 + c;
            buf[e] = make_cpx(a1[gi], a2[gi]);
        }
    }
    __syncthreads();
    lds_fft<T, LOGN, W, NT, W, 1, true, false>(buf, tw);
    cpx<T>* out = C + (long long)b * N * N;
    for (int e = threadIdx.x; e < N * W; e += NT) {
        const int y = e / W, c = e % W;
        out[(long long)y * N + x0 + c] = buf[e];
    }
}

// ---- P2: rows: forward FFT along x, multiply by conj(D)/n^2, inverse ---------
template <typename T, int LOGN>
__global__ void __launch_bounds__((RowCfg<T, LOGN>::NT))
k_ks_rows_generic(cpx<T>* __restrict__ C, const cpx<T>* __restrict__ tw) {
    using Cfg = RowCfg<T, LOGN>;
    constexpr int N = Cfg::N, NT = Cfg::NT, ROWS = Cfg::ROWS;
    __shared__ cpx<T> buf[ROWS * N];
    const int b = blockIdx.y;
    const int y0 = blockIdx.x * ROWS;
    cpx<T>* base = C + (long long)b * N * N + (long long)y0 * N;
    for (int e = threadIdx.x; e < ROWS * N; e += NT) buf[e] = base[e];
    __syncthreads();
    lds_fft<T, LOGN, ROWS, NT, 1, N, false, false>(buf, tw);
    const T inv_n2 = (T)1 / ((T)N * (T)N);
    for (int e = threadIdx.x; e < ROWS * N; e += NT) {
        const int m1 = signed_freq(e % N, N);
        const int m2 = signed_freq(y0 + e / N, N);
        const int den = m1 * m1 + m2 * m2;
        cpx<T> v = buf[e];
        if (den == 0) {
            v = make_cpx((T)0, (T)0);
        } else {
            // conj(D) with D = [(m1^2 - m2^2) + 2 i nu m1 m2] / (m1^2 + m2^2)
            const bool nyq = (m1 == -N / 2) || (m2 == -N / 2);
            const T dr = (T)(m1 * m1 - m2 * m2) / (T)den;
            const T di = nyq ? (T)0 : (T)(2 * m1 * m2) / (T)den;
            v = make_cpx((v.x * dr + v.y * di) * inv_n2, (v.y * dr - v.x * di) * inv_n2);
        }
        buf[e] = v;
    }
    __syncthreads();
    lds_fft<T, LOGN, ROWS, NT, 1, N, false, true>(buf, tw);
    for (int e = threadIdx.x; e < ROWS * N; e += NT) base[e] = buf[e];
}

// ---- P3: inverse FFT along y, split real/imaginary ---------------------------
template <typename T, int LOGN>
__global__ void __launch_bounds__((StripCfg<T, LOGN>::NT))
k_ks_cols_inv_generic(const cpx<T>* __restrict__ C, T* __restrict__ kE, T* __restrict__ kB,
              long long out_stride, const long long* __restrict__ kE_off, const cpx<T>* __restrict__ tw) {
    using Cfg = StripCfg<T, LOGN>;
    constexpr int N = Cfg::N, W = Cfg::W, NT = Cfg::NT;
    __shared__ cpx<T> buf[N * W];
    const int b = blockIdx.y;
    const int x0 = blockIdx.x * W;
    const cpx<T>* in = C + (long long)b * N * N;
    for (int e = threadIdx.x; e < N * W; e += NT) {
        const int y = e / W, c = e % W;
        buf[e] = in[(long long)y * N + x0 + c];
    }
    __syncthreads();
    lds_fft<T, LOGN, W, NT, W, 1, true, true>(buf, tw);
    T* oe = kE + (kE_off ? kE_off[b] : (long long)b * out_stride);
    T* ob = kB ? kB + (long long)b * out_stride : nullptr;
    for (int e = threadIdx.x; e < N * W; e += NT) {
        const int y = e / W, c = e % W;
        const long long gi = (long long)y * N + x0 + c;
        oe[gi] = buf[e].x;
        if (ob) ob[gi] = buf[e].y;
    }
}

// exp(-+2 pi i e / N) from the 4096-entry table
template <typename T, int LOGN, bool INV>
__device__ __forceinline__ cpx<T> table_twiddle(const cpx<T>* __restrict__ tw, int e) {
    const cpx<T> w = tw[(e & ((1 << LOGN) - 1)) << (kMaxLogN - LOGN)];
    return INV ? make_cpx(w.x, -w.y) : w;
}

// exp(-+2 pi i base k / N) for k = 1 .. K-1, passed to f(k, w) in increasing
// k: five table reads (base times 1, 2, 4, 8, 16) and one complex product
// per power, w(k) = w(k without its lowest set bit) * w(lowest set bit), so
// each power carries at most four roundings and only a few are live at once.
template <typename T, int LOGN, bool INV, int K, typename Fn>
__device__ __forceinline__ void twiddle_powers(const cpx<T>* __restrict__ tw, int base, Fn&& f) {
    static_assert(K <= 64, "at most 64 powers");
    constexpr int NB = K <= 2 ? 1 : (K <= 4 ? 2 : (K <= 8 ? 3 : (K <= 16 ? 4 : (K <= 32 ? 5 : 6))));
    cpx<T> p[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) p[b] = table_twiddle<T, LOGN, INV>(tw, base << b);
    cpx<T> w[K];
#pragma unroll
    for (int k = 1; k < K; ++k) {
        const int low = k & -k, rest = k - low;
        const int bit = __builtin_ctz(low);
        w[k] = rest ? cmul(w[rest], p[bit]) : p[bit];
        f(k, w[k]);
    }
}

// Four-step factors: N = N1 * N2, N1 = N2 or 2 N2.
template <int LOGN>
struct FS {
    static constexpr int N = 1 << LOGN;
    static constexpr int N1 = 1 << ((LOGN + 1) / 2);
    static constexpr int N2 = 1 << (LOGN / 2);
    static constexpr int RR = N1 / N2;
};

// Threads and LDS of the four-step column kernels: strips of W columns, N2
// threads per column; WREQ (if smaller) narrows the strip so that a small
// batch still spreads over many workgroups.  A strip's N x W values pass
// through LDS in PH phases of N / PH rows (loads) and N1 / PH first-step
// outputs (exchange).
//   forward (FWD): up to 16 columns and 512 threads.  Where a thread's
//     first-step DFT fits half the register file (FP32, N1 <= 32) the
//     phases keep LDS at 64 KiB and the kernel is built for two workgroups
//     per CU; otherwise LDS is held to 128 KiB at one workgroup per CU;
//   inverse: as many columns (up to 16) as 128 KiB of LDS holds in one
//     phase.  Its first step loads straight from memory and keeps many
//     values in flight, so neither a register cap nor narrower phases pay.
template <typename T, int LOGN, bool FWD, int WREQ = 0>
struct Strip4 {
    static constexpr int N = 1 << LOGN, N1 = FS<LOGN>::N1, N2 = FS<LOGN>::N2;
    static constexpr int CPX = (int)sizeof(cpx<T>);
    static constexpr int WT = 512 / N2 > 16 ? 16 : 512 / N2;
    static constexpr int WL = (128 * 1024 / CPX) / N > 16 ? 16 : (128 * 1024 / CPX) / N;
    static constexpr int WMAX = FWD ? WT : WL;
    static constexpr int W = (WREQ > 0 && WREQ < WMAX) ? WREQ : WMAX;
    static constexpr int NT = W * N2;
    static constexpr bool TWO = FWD && sizeof(T) == 4 && N1 <= 32 && NT >= 256;
    static constexpr int CAP = TWO ? 64 * 1024 : 128 * 1024;
    static constexpr int BYTES = N * W * CPX;
    static constexpr int PH0 = BYTES <= CAP ? 1 : BYTES / CAP;
    static constexpr int PH = PH0 > N1 ? N1 : PH0;
    static constexpr int LDS = N * W / PH;  // complex values
    static constexpr int MINW = TWO ? 2 * NT / 256 : 1;  // waves per SIMD for two workgroups
    static_assert(N1 % PH == 0, "phases split the first-step index evenly");
};
template <typename T, int LOGN, int WREQ = 0>
using StripF = Strip4<T, LOGN, true, WREQ>;
template <typename T, int LOGN, int WREQ = 0>
using StripI = Strip4<T, LOGN, false, WREQ>;

// Strip s and map b of the column kernels' workgroup.  With `xcd` set,
// workgroups are renumbered so that consecutive strips of a map run on one
// XCD (the hardware deals workgroups out to the eight XCDs in turn): strips
// whose row segments share a cache line then meet in one L2 instead of each
// XCD fetching the whole line.  Not used where all maps read one shared
// input (noise realisations), which each XCD keeps in its L2 as it is.
__device__ __forceinline__ void strip_of(int xcd, int& s, int& b) {
    s = blockIdx.x;
    b = blockIdx.y;
    const int nx = gridDim.x;
    const int total = nx * gridDim.y;
    if (xcd && (total & 7) == 0) {
        const int l = blockIdx.x + nx * blockIdx.y;
        const int v = (l & 7) * (total >> 3) + (l >> 3);
        s = v % nx;
        b = v / nx;
    }
}
template <typename T, int LOGN>
struct Row4 {
    static constexpr int N2 = FS<LOGN>::N2, N1 = FS<LOGN>::N1;
    static constexpr int N = 1 << LOGN;
    static constexpr int NT = 128;
    static constexpr int LINES0 = NT / N2 > 0 ? NT / N2 : 1;
    static constexpr int LINES = LINES0 > N ? N : LINES0;
    // exchange region per line: forward [N1][N2+1], inverse [N2][N1+1]
    static constexpr int EX = (N1 * (N2 + 1)) > (N2 * (N1 + 1)) ? (N1 * (N2 + 1)) : (N2 * (N1 + 1));
};

// Orders the LDS accesses of one wavefront (the lanes of one transform).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// ---- P1: load shears (optionally rotate), forward FFT along y (four-step) -------
template <typename T, int LOGN, bool ROTATE, int WREQ>
__global__ void __launch_bounds__((StripF<T, LOGN, WREQ>::NT), (StripF<T, LOGN, WREQ>::MINW))
k_ks_cols_fwd(const T* __restrict__ g1, const T* __restrict__ g2, long long g_stride,
              const long long* __restrict__ g1_off, const long long* __restrict__ g2_off,
              cpx<T>* __restrict__ C, uint64_t seed, uint64_t r0, const cpx<T>* __restrict__ tw,
              int xcd) {
    using F = FS<LOGN>;
    using S = StripF<T, LOGN, WREQ>;
    constexpr int N = F::N, N1 = F::N1, N2 = F::N2, W = S::W, NT = S::NT, PH = S::PH;
    constexpr int ROWS = N / PH, K = N1 / PH;  // rows and first-step indices per phase
    __shared__ cpx<T> buf[S::LDS];
    int sx, b;
    strip_of(xcd, sx, b);
    const int x0 = sx * W;
    const T* a1 = g1 + (g1_off ? g1_off[b] : (long long)b * g_stride);
    const T* a2 = g2 + (g2_off ? g2_off[b] : (long long)b * g_stride);
    constexpr int G = 16 / (int)sizeof(T);  // values per 16-byte load
    const int c = threadIdx.x % W, t = threadIdx.x / W;
    // row y = N2 n1 + t of column c goes to a[n1]; phase p stages rows
    // p ROWS .. (p+1) ROWS - 1, i.e. n1 = p K .. (p+1) K - 1
    cpx<T> a[N1];
#pragma unroll
    for (int p = 0; p < PH; ++p) {
        const int y0 = p * ROWS;
        if (p > 0) __syncthreads();  // the previous phase's reads are done
        if (ROTATE) {
            // one Philox block covers 8 consecutive pixels of a row
            constexpr int OCT_PER_ROW = (W + 7) / 8;
            const uint64_t r = r0 + b;
            for (int o = threadIdx.x; o < ROWS * OCT_PER_ROW; o += NT) {
                const int yl = o / OCT_PER_ROW, y = y0 + yl;
                const int cx = (o % OCT_PER_ROW) * 8;
                const int xa = (W >= 8) ? (x0 + cx) : (x0 & ~7);
                const uint64_t pix = (uint64_t)y * N + xa;
                uint32_t u[8];
                philox_block_u32(seed, r, pix >> 3, u);
                T gp[8], gq[8];
                load16<T, 8>(a1 + (long long)y * N + xa, gp);
                load16<T, 8>(a2 + (long long)y * N + xa, gq);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int x = xa + i;
                    if (W < 8 && (x < x0 || x >= x0 + W)) continue;
                    rotate_by_u32(u[i], gp[i], gq[i]);
                    buf[yl * W + (x - x0)] = make_cpx(gp[i], gq[i]);
                }
            }
        } else {
            // G consecutive columns of a row per load
            for (int e = threadIdx.x; e < ROWS * (W / G); e += NT) {
                const int yl = e / (W / G), cc = (e % (W / G)) * G;
                const long long gi = (long long)(y0 + yl) * N + x0 + cc;
                T gp[G], gq[G];
                load16<T, G>(a1 + gi, gp);
                load16<T, G>(a2 + gi, gq);
#pragma unroll
                for (int i = 0; i < G; ++i) buf[yl * W + cc + i] = make_cpx(gp[i], gq[i]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int n1 = 0; n1 < K; ++n1) a[p * K + n1] = buf[(N2 * n1 + t) * W + c];
    }
    dft_reg<T, N1, false>(a);
    twiddle_powers<T, LOGN, false, N1>(tw, t, [&](int k1, const cpx<T>& w) { a[k1] = cmul(a[k1], w); });
    cpx<T>* out = C + (long long)b * N * N + x0 + c;
    // exchange phase q: first-step outputs k1 = q K .. (q+1) K - 1, then the
    // second step over n2 for each (k1, column) of the phase
#pragma unroll
    for (int q = 0; q < PH; ++q) {
        __syncthreads();  // LDS free
#pragma unroll
        for (int kl = 0; kl < K; ++kl) buf[(kl * N2 + t) * W + c] = a[q * K + kl];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < (K + N2 - 1) / N2; ++r) {
            const int kl = t + N2 * r;
            if (K % N2 == 0 || kl < K) {
                cpx<T> v[N2];
#pragma unroll
                for (int n2 = 0; n2 < N2; ++n2) v[n2] = buf[(kl * N2 + n2) * W + c];
                dft_reg<T, N2, false>(v);
                const int k1 = q * K + kl;
#pragma unroll
                for (int k2 = 0; k2 < N2; ++k2) store_stream(&out[(long long)(k1 + N1 * k2) * N], v[k2]);
            }
        }
    }
}

// ---- P2: rows: forward FFT along x, multiply by conj(D)/n^2, inverse (four-step) -
// The forward transform of one row for the N2 lanes t of a line, with E its
// exchange region: on return b[r][k2] holds the row's transform at
// frequency k1 + N1 k2, k1 = t + N2 r.
template <typename T, int LOGN>
__device__ __forceinline__ void ks_row_spectrum(const cpx<T>* __restrict__ row, int t, cpx<T>* E,
                                                const cpx<T>* __restrict__ tw,
                                                cpx<T> (&b)[FS<LOGN>::RR][FS<LOGN>::N2]) {
    using F = FS<LOGN>;
    constexpr int N1 = F::N1, N2 = F::N2, RR = F::RR;
    cpx<T> a[N1];
    // forward, step 1: DFT_N1 over n1 of x[N2 n1 + t]
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) a[n1] = row[N2 * n1 + t];
    dft_reg<T, N1, false>(a);
    E[t] = a[0];
    twiddle_powers<T, LOGN, false, N1>(tw, t, [&](int k1, const cpx<T>& w) {
        E[k1 * (N2 + 1) + t] = cmul(a[k1], w);
    });
    wave_lds_sync();
    // forward, step 2: DFT_N2 over n2 -> X[k1 + N1 k2], k1 = t + N2 r
#pragma unroll
    for (int r = 0; r < RR; ++r) {
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) b[r][n2] = E[(t + N2 * r) * (N2 + 1) + n2];
        dft_reg<T, N2, false>(b[r]);
    }
}

// b (laid out as ks_row_spectrum leaves it, spectral row y) times
// conj(D)/(SCALE_DEN n^2), with D = [(m1^2 - m2^2) + 2 i nu m1 m2] / (m1^2 + m2^2).
    // Every integer here is exact in T (|m| <= n/2, so m1^2 + m2^2 < 2^24),
    // so the arithmetic runs in T without integer multiplies; 1 / max(den, 1)
    // gives D(0) = 0 because both numerators vanish there.  The imaginary
    // part is 0 on the Nyquist row and column.  The frequency index is
    // t + c with c = N2 r + N1 k2 a multiple of N2 and t < N2, so it lies
    // below n/2 exactly when c does: m1 is t plus a constant.
template <typename T, int LOGN, int SCALE_DEN>
__device__ __forceinline__ void ks_multiply(cpx<T> (&b)[FS<LOGN>::RR][FS<LOGN>::N2], int y, int t) {
    using F = FS<LOGN>;
    constexpr int N = F::N, N1 = F::N1, N2 = F::N2, RR = F::RR;
    const T scale = (T)1 / ((T)N * (T)N * (T)SCALE_DEN);
    const int m2i = signed_freq(y, N);
    const T m2 = (T)m2i, m2sq = m2 * m2;
    const T two_m2 = m2i == -N / 2 ? (T)0 : (T)2 * m2;
    const T tf = (T)t;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
            const int c = N2 * r + N1 * k2;
            const T m1 = tf + (T)(c < N / 2 ? c : c - N);
            const T m1sq = m1 * m1;
            const T s = scale * recip(fmax(m1sq + m2sq, (T)1));
            const T dr = (m1sq - m2sq) * s;
            const T di = (c == N / 2 && t == 0) ? (T)0 : (m1 * two_m2) * s;
            const cpx<T> v = b[r][k2];
            b[r][k2] = make_cpx(v.x * dr + v.y * di, v.y * dr - v.x * di);
        }
    }
}

// The forward half of one spectral row y: transform, then times
// conj(D)/(SCALE_DEN n^2).
template <typename T, int LOGN, int SCALE_DEN = 1>
__device__ __forceinline__ void ks_row_forward(const cpx<T>* __restrict__ row, int y, int t,
                                               cpx<T>* E, const cpx<T>* __restrict__ tw,
                                               cpx<T> (&b)[FS<LOGN>::RR][FS<LOGN>::N2]) {
    ks_row_spectrum<T, LOGN>(row, t, E, tw, b);
    ks_multiply<T, LOGN, SCALE_DEN>(b, y, t);
}

// The inverse half: from b[r][k2] at frequency k1 + N1 k2 (k1 = t + N2 r),
// on return a[n] holds the row's inverse transform at x = t + N2 n.
template <typename T, int LOGN>
__device__ __forceinline__ void ks_row_inverse(cpx<T> (&b)[FS<LOGN>::RR][FS<LOGN>::N2], int t,
                                               cpx<T>* E, const cpx<T>* __restrict__ tw,
                                               cpx<T> (&a)[FS<LOGN>::N1]) {
    using F = FS<LOGN>;
    constexpr int N1 = F::N1, N2 = F::N2, RR = F::RR;
    wave_lds_sync();  // earlier reads of the exchange region are done before it is reused
    // inverse, step 1: DFT_N2 over k2 for each k1 held, twiddle, exchange
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int k1 = t + N2 * r;
        dft_reg<T, N2, true>(b[r]);
        E[k1] = b[r][0];
        twiddle_powers<T, LOGN, true, N2>(tw, k1, [&](int m, const cpx<T>& w) {
            E[m * (N1 + 1) + k1] = cmul(b[r][m], w);
        });
    }
    wave_lds_sync();
    // inverse, step 2: DFT_N1 over k1 for m = t -> x[t + N2 n]
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) a[k1] = E[t * (N1 + 1) + k1];
    dft_reg<T, N1, true>(a);
}

// The whole row: forward, multiply, inverse.
template <typename T, int LOGN>
__device__ __forceinline__ void ks_row_line(const cpx<T>* __restrict__ row, int y, int t,
                                            cpx<T>* E, const cpx<T>* __restrict__ tw,
                                            cpx<T> (&a)[FS<LOGN>::N1]) {
    cpx<T> b[FS<LOGN>::RR][FS<LOGN>::N2];
    ks_row_forward<T, LOGN>(row, y, t, E, tw, b);
    ks_row_inverse<T, LOGN>(b, t, E, tw, a);
}

template <typename T, int LOGN>
__global__ void __launch_bounds__((Row4<T, LOGN>::NT))
k_ks_rows(cpx<T>* __restrict__ C, const cpx<T>* __restrict__ tw) {
    using F = FS<LOGN>;
    using R4 = Row4<T, LOGN>;
    constexpr int N = F::N, N1 = F::N1, N2 = F::N2;
    __shared__ cpx<T> ex[R4::LINES * R4::EX];
    const int line = threadIdx.x / N2, t = threadIdx.x % N2;
    if (line >= R4::LINES) return;  // no workgroup barrier follows
    const int y = blockIdx.x * R4::LINES + line;
    cpx<T>* row = C + (long long)blockIdx.y * N * N + (long long)y * N;
    cpx<T> a[N1];
    ks_row_line<T, LOGN>(row, y, t, ex + line * R4::EX, tw, a);
#pragma unroll
    for (int n = 0; n < N1; ++n) row[t + N2 * n] = a[n];
}

// P2 for pairs of maps whose kappa_B is not wanted.  kappa_E of a map is
// the inverse transform of the Hermitian part H(k) = [K(k) + conj(K(-k))]/2
// of its spectrum K, which is real; two maps a, b then share one inverse
// transform, of Z = H_a + i H_b, whose real and imaginary parts are their
// kappa_E.  A workgroup unit takes spectral rows y and -y (rows 0 and n/2
// are their own partners) of both maps: four lines, one per (map, row),
// run the forward transform and the multiply and leave their spectral rows
// in LDS in natural frequency order (-k is the mirrored address).  The two
// Z rows, y and -y, are then transformed back by two lane groups of 2 N2
// lanes each (the lanes of map a, then those of map b), so every lane does
// the same work: within a group the low half holds the even-indexed and the
// high half the odd-indexed inputs of each length-N2 and length-N1 DFT of
// the four-step inverse, and one radix-2 step across the halves completes
// them.  The group writes its Z row over map a's row.  Pair p holds maps 2p
// and 2p+1 (map 2p alone, read twice, if 2p+1 = batch).
template <typename T, int LOGN>
struct RowPair {
    static constexpr int N2 = FS<LOGN>::N2, N = 1 << LOGN;
    static constexpr int U0 = 128 / (4 * N2) > 0 ? 128 / (4 * N2) : 1;
    static constexpr int UNITS = U0 > N / 2 ? N / 2 : U0;  // row pairs per workgroup
    static constexpr int NT = UNITS * 4 * N2;
};

// Exchange across the halves of a group of 2 H lanes (H a power of two, the
// group aligned to 2 H): afterwards a low lane holds (its d, its partner's
// d) and a high lane (its partner's s, its s) in (d, s).
template <int H>
__device__ __forceinline__ void half_swap_u32(uint32_t& d, uint32_t& s, bool hi) {
    if constexpr (H == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(d, s, false, false);
        d = r[0];
        s = r[1];
    } else if constexpr (H == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(d, s, false, false);
        d = r[0];
        s = r[1];
    } else {
        const uint32_t got = (uint32_t)__shfl_xor((int)(hi ? d : s), H);
        if (hi) d = got;
        else s = got;
    }
}
template <int H, typename T>
__device__ __forceinline__ void half_swap(T& d, T& s, bool hi) {
    if constexpr (sizeof(T) == 4) {
        uint32_t a = __builtin_bit_cast(uint32_t, d), b = __builtin_bit_cast(uint32_t, s);
        half_swap_u32<H>(a, b, hi);
        d = __builtin_bit_cast(T, a);
        s = __builtin_bit_cast(T, b);
    } else {
        const uint64_t a = __builtin_bit_cast(uint64_t, d), b = __builtin_bit_cast(uint64_t, s);
        uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32), bl = (uint32_t)b, bh = (uint32_t)(b >> 32);
        half_swap_u32<H>(al, bl, hi);
        half_swap_u32<H>(ah, bh, hi);
        d = __builtin_bit_cast(T, ((uint64_t)ah << 32) | al);
        s = __builtin_bit_cast(T, ((uint64_t)bh << 32) | bl);
    }
}

// Radix-2 step of an inverse length-2M DFT across a lane pair, from the
// half-length DFTs E (low lane) and O (high lane) after half_swap: the lane
// of half h forms X[I + h M/2] = E + w O and X[I + h M/2 + M] = E - w O with
// w = exp(2 pi i (I + h M/2) / 2M), which is i times the low lane's twiddle.
template <typename T, int L, int I>
__device__ __forceinline__ void pair_bfly(cpx<T>& e, cpx<T>& o, bool hi) {
    constexpr CS w = cos_sin_2pi(I, L);
    const T wr = hi ? (T)-w.s : (T)w.c;
    const T wi = hi ? (T)w.c : (T)w.s;
    const T xr = fma(wr, o.x, fma(-wi, o.y, e.x));
    const T xi = fma(wr, o.y, fma(wi, o.x, e.y));
    o = make_cpx<T>(fma((T)2, e.x, -xr), fma((T)2, e.y, -xi));
    e = make_cpx<T>(xr, xi);
}
template <typename T, int M, int H, int... I>
__device__ __forceinline__ void pair_bflies(cpx<T> (&v)[M], bool hi, std::integer_sequence<int, I...>) {
    constexpr int Q = M / 2;
    ((half_swap<H>(v[I].x, v[Q + I].x, hi), half_swap<H>(v[I].y, v[Q + I].y, hi)), ...);
    (pair_bfly<T, 2 * M, I>(v[I], v[Q + I], hi), ...);
}
// Inverse DFT of length 2M over a lane pair (l, l + H): the low lane holds
// inputs 0, 2, .., the high lane 1, 3, .. (M each, in order).  On return the
// lane of half h holds outputs i + h M/2 in v[i] and i + h M/2 + M in
// v[M/2 + i], i < M/2.
template <typename T, int M, int H>
__device__ __forceinline__ void pair_dft_inv(cpx<T> (&v)[M], bool hi) {
    static_assert(M >= 2, "at least two values per lane");
    dft_reg<T, M, true>(v);
    pair_bflies<T, M, H>(v, hi, std::make_integer_sequence<int, M / 2>{});
}
// The output index held in v[j] by the lane of half h after pair_dft_inv.
template <int M>
__device__ __forceinline__ constexpr int pair_out(int j, int h) {
    return j < M / 2 ? j + h * (M / 2) : j - M / 2 + h * (M / 2) + M;
}

// ks_multiply for a lane pair (t, t + N2) holding spectral rows y0 (low
// half) and -y0 (high half), 0 < y0 < n/2, at the same frequencies.  conj(D)
// of row -y0 is the conjugate of that of row y0, so each half evaluates it,
// with y0's sign, at half of the frequencies (the low half at k2 < N2/2,
// the high half at k2 + N2/2) and the halves exchange the values; passing
// (V, -V) for the imaginary part hands each half its own row's sign.  The
// factors are those ks_multiply computes, value for value (the sign changes
// are exact).
template <typename T, int LOGN, int SCALE_DEN>
__device__ __forceinline__ void ks_multiply_pair(cpx<T> (&b)[FS<LOGN>::RR][FS<LOGN>::N2], int y0, int t,
                                                 bool hi) {
    using F = FS<LOGN>;
    constexpr int N = F::N, N1 = F::N1, N2 = F::N2, RR = F::RR, HALF = N2 / 2;
    const T scale = (T)1 / ((T)N * (T)N * (T)SCALE_DEN);
    const T m2 = (T)y0, m2sq = m2 * m2, two_m2 = (T)2 * m2;
    // the high half's frequency index is t + c + n/2 with c = N2 r + N1 k2 < n/2,
    // so its m1 is t - n/2 + c
    const T tb = (T)t - (hi ? (T)(N / 2) : (T)0);
    const auto apply = [](cpx<T>& v, T dr, T di) {
        v = make_cpx(v.x * dr + v.y * di, v.y * dr - v.x * di);
    };
#pragma unroll
    for (int r = 0; r < RR; ++r) {
#pragma unroll
        for (int k2 = 0; k2 < HALF; ++k2) {
            const int c = N2 * r + N1 * k2;
            const T m1 = tb + (T)c;
            const T m1sq = m1 * m1;
            const T s = scale * recip(fmax(m1sq + m2sq, (T)1));
            T dr_lo = (m1sq - m2sq) * s, dr_hi = dr_lo;
            // the Nyquist column n/2 is the high half's c = 0 at t = 0
            const T v = (c == 0 && hi && t == 0) ? (T)0 : (m1 * two_m2) * s;
            T di_lo = v, di_hi = -v;
            half_swap<N2>(dr_lo, dr_hi, hi);
            half_swap<N2>(di_lo, di_hi, hi);
            apply(b[r][k2], dr_lo, di_lo);
            apply(b[r][k2 + HALF], dr_hi, di_hi);
        }
    }
}

template <typename T, int LOGN>
__global__ void __launch_bounds__((RowPair<T, LOGN>::NT))
k_ks_rows_pair(cpx<T>* __restrict__ C, int batch, const cpx<T>* __restrict__ tw) {
    using F = FS<LOGN>;
    using RP = RowPair<T, LOGN>;
    constexpr int N = F::N, N1 = F::N1, N2 = F::N2, RR = F::RR, EX = Row4<T, LOGN>::EX;
    constexpr int M2 = N2 / 2, M1 = N1 / 2;  // values per lane in the two inverse steps
    // a lane group (2 N2 lanes, aligned) lies in one wavefront, so wave-level
    // ordering covers its exchange and its cross-lane steps
    static_assert(2 * N2 <= 64, "a lane group must lie in one wavefront");
    static_assert(N2 >= 4, "at least two values per lane and half");
    __shared__ cpx<T> ex[RP::UNITS * 4 * EX];
    const int line = threadIdx.x / N2, t = threadIdx.x % N2;
    const int u = line >> 2, role = line & 3;  // role: map (role >> 1), row (role & 1)
    const int q = blockIdx.x * RP::UNITS + u;
    const int r0 = q, r1 = q == 0 ? N / 2 : N - q;
    const int ma = 2 * blockIdx.y;
    const int mb = ma + 1 < batch ? ma + 1 : ma;
    {
        const int y = (role & 1) ? r1 : r0;
        const cpx<T>* row = C + (long long)((role >> 1) ? mb : ma) * N * N + (long long)y * N;
        cpx<T>* E = ex + line * EX;
        cpx<T> b[RR][N2];
        ks_row_spectrum<T, LOGN>(row, t, E, tw, b);
        // times conj(D), carrying the 1/2 of H; rows 0 and n/2 are not a
        // conjugate pair
        if (q != 0) ks_multiply_pair<T, LOGN, 2>(b, r0, t, (role & 1) != 0);
        else ks_multiply<T, LOGN, 2>(b, y, t);
        wave_lds_sync();  // the forward exchange's reads are done
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) E[t + N2 * r + N1 * k2] = b[r][k2];
    }
    // inverse: group g = role >> 1 transforms Z row y_g (slot g); h = role & 1
    const int g = role >> 1, h = role & 1;
    const bool hi = h != 0;
    const int yg = g ? r1 : r0;
    const int pg = q == 0 ? g : 1 - g;  // slot of row -y_g
    // inter-step twiddles exp(2 pi i k1 m / N) for this lane's k1 and m
    cpx<T> w[RR][M2];
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int j = 0; j < M2; ++j) w[r][j] = table_twiddle<T, LOGN, true>(tw, (t + N2 * r) * pair_out<M2>(j, h));
    __syncthreads();  // the four spectral rows of every unit are in LDS (and C's rows read)
    // Z = H_a + i H_b at k1 = t + N2 r, k2 = 2 j + h (the spectra carry the 1/2)
    const cpx<T>* base = ex + (u * 4) * EX;
    const cpx<T>* Ka = base + g * EX;
    const cpx<T>* Kap = base + pg * EX;
    const cpx<T>* Kb = base + (2 + g) * EX;
    const cpx<T>* Kbp = base + (2 + pg) * EX;
    cpx<T> z[RR][M2];
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int j = 0; j < M2; ++j) {
            const int kx = t + N2 * r + N1 * (2 * j + h), mk = (N - kx) & (N - 1);
            const cpx<T> ka = Ka[kx], kap = Kap[mk], kb = Kb[kx], kbp = Kbp[mk];
            const T har = ka.x + kap.x, hai = ka.y - kap.y;
            const T hbr = kb.x + kbp.x, hbi = kb.y - kbp.y;
            z[r][j] = make_cpx(har - hbi, hai + hbr);
        }
    // step 1: DFT_N2 over k2 for each k1 held, then the twiddle
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        pair_dft_inv<T, M2, N2>(z[r], hi);
#pragma unroll
        for (int j = 0; j < M2; ++j) z[r][j] = cmul(z[r][j], w[r][j]);
    }
    __syncthreads();  // every group's reads of the spectra are done
    cpx<T>* E = ex + (u * 4 + 2 * g) * EX;  // this group's exchange region
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int j = 0; j < M2; ++j) E[pair_out<M2>(j, h) * (N1 + 1) + t + N2 * r] = z[r][j];
    wave_lds_sync();
    // step 2: DFT_N1 over k1 for m = t -> x[t + N2 n]
    cpx<T> v[M1];
#pragma unroll
    for (int j = 0; j < M1; ++j) v[j] = E[t * (N1 + 1) + 2 * j + h];
    pair_dft_inv<T, M1, N2>(v, hi);
    cpx<T>* out = C + (long long)ma * N * N + (long long)yg * N;
#pragma unroll
    for (int j = 0; j < M1; ++j) out[t + N2 * pair_out<M1>(j, h)] = v[j];
}

// ---- P3: inverse FFT along y (four-step), split real/imaginary -----------------
template <typename T, int LOGN, int WREQ>
__global__ void __launch_bounds__((StripI<T, LOGN, WREQ>::NT), (StripI<T, LOGN, WREQ>::MINW))
k_ks_cols_inv(const cpx<T>* __restrict__ C, long long in_stride, T* __restrict__ kE,
              T* __restrict__ kB, long long out_stride, int kB_count,
              const long long* __restrict__ kE_off, const cpx<T>* __restrict__ tw, int xcd) {
    using F = FS<LOGN>;
    using S = StripI<T, LOGN, WREQ>;
    constexpr int N = F::N, N1 = F::N1, N2 = F::N2, W = S::W, PH = S::PH, K = N1 / PH;
    __shared__ cpx<T> buf[S::LDS];
    int sx, b;
    strip_of(xcd, sx, b);
    const int x0 = sx * W;
    const int c = threadIdx.x % W, t = threadIdx.x / W;
    const cpx<T>* in = C + (long long)b * in_stride + x0 + c;
    cpx<T> a[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) a[n1] = in[(long long)(N2 * n1 + t) * N];
    dft_reg<T, N1, true>(a);
    twiddle_powers<T, LOGN, true, N1>(tw, t, [&](int k1, const cpx<T>& w) { a[k1] = cmul(a[k1], w); });
    T* oe = kE + (kE_off ? kE_off[b] : (long long)b * out_stride) + x0 + c;
    T* ob = (kB && b < kB_count) ? kB + (long long)b * out_stride + x0 + c : nullptr;
    // exchange in PH phases of K first-step outputs each, as the forward pass
#pragma unroll
    for (int q = 0; q < PH; ++q) {
        if (q > 0) __syncthreads();  // the previous phase's reads are done
#pragma unroll
        for (int kl = 0; kl < K; ++kl) buf[(kl * N2 + t) * W + c] = a[q * K + kl];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < (K + N2 - 1) / N2; ++r) {
            const int kl = t + N2 * r;
            if (K % N2 == 0 || kl < K) {
                cpx<T> v[N2];
#pragma unroll
                for (int n2 = 0; n2 < N2; ++n2) v[n2] = buf[(kl * N2 + n2) * W + c];
                dft_reg<T, N2, true>(v);
                const int k1 = q * K + kl;
#pragma unroll
                for (int k2 = 0; k2 < N2; ++k2) {
                    const long long gi = (long long)(k1 + N1 * k2) * N;
                    oe[gi] = v[k2].x;
                    if (ob) ob[gi] = v[k2].y;
                }
            }
        }
    }
}

// ---- host launchers ------------------------------------------------------------
// Double-precision transforms from 1024 points keep their data in LDS (their
// per-thread DFTs would not fit the register file); everything else runs the
// four-step register kernels.
template <typename T, int LOGN>
constexpr bool use_generic() { return sizeof(T) == 8 && LOGN >= 10; }

// Pairs of maps share the inverse transform where the four-step kernels run
// and the four exchange rows of a unit fit 128 KiB of LDS (as the row pass's
// four rows do): up to n = 2048 in float32.
template <typename T, int LOGN>
constexpr bool pair_ok() {
    return !use_generic<T, LOGN>() && 2 * FS<LOGN>::N2 <= 64 &&
           (size_t)RowPair<T, LOGN>::UNITS * 4 * Row4<T, LOGN>::EX * sizeof(cpx<T>) <= 128 * 1024;
}

// The four-step kernels with strips of WREQ columns.
template <typename T, int LOGN, int WREQ>
static hipError_t ks_launch_w(const KsArgs<T>& a) {
    constexpr int N = 1 << LOGN;
    using SF = StripF<T, LOGN, WREQ>;
    using SI = StripI<T, LOGN, WREQ>;
    using R = Row4<T, LOGN>;
    const dim3 gf(N / SF::W, a.batch), gi(N / SI::W, a.batch), gr(N / R::LINES, a.batch);
    // XCD grouping where strips read or write row segments narrower than a
    // 128-byte line, except for a shared input (noise realisations)
    const bool shared_in = a.g_stride == 0 && !a.g1_off && a.batch > 1;
    const int xcd_in = (!shared_in && SF::W * (int)sizeof(T) < 128) ? 1 : 0;
    const int xcd_out = SI::W * (int)sizeof(T) < 128 ? 1 : 0;
    if (a.rotate)
        AMAP_LAUNCH("ks_cols_fwd_rotate", a.stream,
                    k_ks_cols_fwd<T, LOGN, true, WREQ><<<gf, SF::NT, 0, a.stream>>>(
                        a.g1, a.g2, a.g_stride, a.g1_off, a.g2_off, a.C, a.seed, a.r0, a.tw, xcd_in));
    else
        AMAP_LAUNCH("ks_cols_fwd", a.stream,
                    k_ks_cols_fwd<T, LOGN, false, WREQ><<<gf, SF::NT, 0, a.stream>>>(
                        a.g1, a.g2, a.g_stride, a.g1_off, a.g2_off, a.C, a.seed, a.r0, a.tw, xcd_in));
    if constexpr (pair_ok<T, LOGN>()) {
        if (a.pair_e) {
            using RP = RowPair<T, LOGN>;
            if (a.kE_off || a.batch < 1) return hipErrorInvalidValue;
            const int pairs = (a.batch + 1) / 2;
            AMAP_LAUNCH("ks_rows_pair", a.stream,
                        k_ks_rows_pair<T, LOGN><<<dim3((N / 2) / RP::UNITS, pairs), RP::NT, 0, a.stream>>>(
                            a.C, a.batch, a.tw));
            AMAP_LAUNCH("ks_cols_inv_pair", a.stream,
                        k_ks_cols_inv<T, LOGN, WREQ><<<dim3(N / SI::W, pairs), SI::NT, 0, a.stream>>>(
                            a.C, 2ll * N * N, a.kE, a.kE + a.out_stride, 2 * a.out_stride,
                            a.batch / 2, nullptr, a.tw, xcd_out));
            return hipGetLastError();
        }
    }
    AMAP_LAUNCH("ks_rows", a.stream, k_ks_rows<T, LOGN><<<gr, R::NT, 0, a.stream>>>(a.C, a.tw));
    AMAP_LAUNCH("ks_cols_inv", a.stream,
                k_ks_cols_inv<T, LOGN, WREQ><<<gi, SI::NT, 0, a.stream>>>(
                    a.C, (long long)N * N, a.kE, a.pair_e ? nullptr : a.kB, a.out_stride, a.batch,
                    a.kE_off, a.tw, xcd_out));
    return hipGetLastError();
}

template <typename T, int LOGN>
static hipError_t ks_launch_n(const KsArgs<T>& a) {
    constexpr int N = 1 << LOGN;
    if constexpr (use_generic<T, LOGN>()) {
        using S = StripCfg<T, LOGN>;
        using R = RowCfg<T, LOGN>;
        const dim3 gs(N / S::W, a.batch), gr(N / R::ROWS, a.batch);
        if (a.rotate)
            AMAP_LAUNCH("ks_cols_fwd_rotate", a.stream,
                        k_ks_cols_fwd_generic<T, LOGN, true><<<gs, S::NT, 0, a.stream>>>(
                            a.g1, a.g2, a.g_stride, a.g1_off, a.g2_off, a.C, a.seed, a.r0, a.tw));
        else
            AMAP_LAUNCH("ks_cols_fwd", a.stream,
                        k_ks_cols_fwd_generic<T, LOGN, false><<<gs, S::NT, 0, a.stream>>>(
                            a.g1, a.g2, a.g_stride, a.g1_off, a.g2_off, a.C, a.seed, a.r0, a.tw));
        AMAP_LAUNCH("ks_rows", a.stream,
                    k_ks_rows_generic<T, LOGN><<<gr, R::NT, 0, a.stream>>>(a.C, a.tw));
        AMAP_LAUNCH("ks_cols_inv", a.stream,
                    k_ks_cols_inv_generic<T, LOGN><<<gs, S::NT, 0, a.stream>>>(a.C, a.kE, a.kB,
                                                                                a.out_stride, a.kE_off, a.tw));
    } else {
        // strip width: the widest unless the batch is too small to give the
        // column passes ~512 workgroups at it; then narrower strips, down to
        // 4 columns, from n = 256 (each pass caps the request at its own
        // widest strip)
        constexpr int WMAX = StripF<T, LOGN>::W > StripI<T, LOGN>::W ? StripF<T, LOGN>::W
                                                                     : StripI<T, LOGN>::W;
        int w = WMAX;
        while (N >= 256 && w > 4 && (long long)(N / w) * a.batch < 512) w /= 2;
        if constexpr (WMAX >= 16) {
            if (w == 16) return ks_launch_w<T, LOGN, 16>(a);
        }
        if constexpr (WMAX >= 8) {
            if (w == 8) return ks_launch_w<T, LOGN, 8>(a);
        }
        return ks_launch_w<T, LOGN, 4>(a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ks(const KsArgs<T>& a) {
    switch (a.logn) {
        case 4: return ks_launch_n<T, 4>(a);
        case 5: return ks_launch_n<T, 5>(a);
        case 6: return ks_launch_n<T, 6>(a);
        case 7: return ks_launch_n<T, 7>(a);
        case 8: return ks_launch_n<T, 8>(a);
        case 9: return ks_launch_n<T, 9>(a);
        case 10: return ks_launch_n<T, 10>(a);
        case 11: return ks_launch_n<T, 11>(a);
        case 12: return ks_launch_n<T, 12>(a);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_ks<float>(const KsArgs<float>&);
template hipError_t launch_ks<double>(const KsArgs<double>&);

}  // namespace amap

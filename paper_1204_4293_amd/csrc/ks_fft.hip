// Kaiser-Squires inversion on the GPU: a two-dimensional complex FFT built
// from LDS-resident Stockham radix-4 (+ one radix-2) passes, with the
// spectral multiply by conj(D(k)) fused into the row pass.
//
// Pass structure for one n x n map (columns first, so that the row pass sees
// whole spectral rows and can apply the KS kernel between its forward and
// inverse transforms):
//   P1  column strips:  (g1 + i g2) [optionally rotated by Philox phases]
//                       -> forward FFT along y             -> C
//   P2  whole rows:     forward FFT along x, multiply by conj(D)/n^2,
//                       inverse FFT along x                -> C
//   P3  column strips:  inverse FFT along y -> kappa_E = Re, kappa_B = Im
// A strip is W adjacent columns held in LDS at full height, so every HBM
// access is a W-element row segment; a row pass holds whole rows.
#include "amap_device.h"
#include "amap_launch.h"

namespace amap {

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

// ---- P1: load shears (optionally rotate), forward FFT along y -------------------
// grid: (n / W strips, batch).  Map b reads g1 + b*g_stride (g_stride = 0 when
// every batch entry is a noise realisation of the same map) and writes
// C + b*n*n.  Realisation index r = r0 + b.
template <typename T, int LOGN, bool ROTATE>
__global__ void __launch_bounds__((StripCfg<T, LOGN>::NT))
k_ks_cols_fwd(const T* __restrict__ g1, const T* __restrict__ g2, long long g_stride,
              cpx<T>* __restrict__ C, uint64_t seed, uint64_t r0,
              const cpx<T>* __restrict__ tw) {
    using Cfg = StripCfg<T, LOGN>;
    constexpr int N = Cfg::N, W = Cfg::W, NT = Cfg::NT;
    __shared__ cpx<T> buf[N * W];
    const int b = blockIdx.y;
    const int x0 = blockIdx.x * W;
    const T* a1 = g1 + (long long)b * g_stride;
    const T* a2 = g2 + (long long)b * g_stride;
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
k_ks_rows(cpx<T>* __restrict__ C, const cpx<T>* __restrict__ tw) {
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
k_ks_cols_inv(const cpx<T>* __restrict__ C, T* __restrict__ kE, T* __restrict__ kB,
              long long out_stride, const cpx<T>* __restrict__ tw) {
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
    T* oe = kE + (long long)b * out_stride;
    T* ob = kB ? kB + (long long)b * out_stride : nullptr;
    for (int e = threadIdx.x; e < N * W; e += NT) {
        const int y = e / W, c = e % W;
        const long long gi = (long long)y * N + x0 + c;
        oe[gi] = buf[e].x;
        if (ob) ob[gi] = buf[e].y;
    }
}

// ---- host launchers ------------------------------------------------------------
template <typename T, int LOGN>
static hipError_t ks_launch_n(const KsArgs<T>& a) {
    using S = StripCfg<T, LOGN>;
    using R = RowCfg<T, LOGN>;
    constexpr int N = 1 << LOGN;
    const dim3 gs(N / S::W, a.batch), gr(N / R::ROWS, a.batch);
    if (a.rotate)
        AMAP_LAUNCH("ks_cols_fwd_rotate", a.stream,
                    k_ks_cols_fwd<T, LOGN, true><<<gs, S::NT, 0, a.stream>>>(
                        a.g1, a.g2, a.g_stride, a.C, a.seed, a.r0, a.tw));
    else
        AMAP_LAUNCH("ks_cols_fwd", a.stream,
                    k_ks_cols_fwd<T, LOGN, false><<<gs, S::NT, 0, a.stream>>>(
                        a.g1, a.g2, a.g_stride, a.C, a.seed, a.r0, a.tw));
    AMAP_LAUNCH("ks_rows", a.stream, k_ks_rows<T, LOGN><<<gr, R::NT, 0, a.stream>>>(a.C, a.tw));
    AMAP_LAUNCH("ks_cols_inv", a.stream,
                k_ks_cols_inv<T, LOGN><<<gs, S::NT, 0, a.stream>>>(a.C, a.kE, a.kB, a.out_stride,
                                                                    a.tw));
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

// In-register DFTs with compile-time twiddles, used by the four-step FFT
// kernels.  Host-callable as well, so the building blocks can be checked on
// the CPU.
#pragma once

#include <utility>

#include "amap_device.h"

namespace amap {

// ---- compile-time twiddles and in-register DFTs -------------------------------
struct CS {
    double c, s;
};
constexpr double kPiD = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
    double t = x, s = x;
    for (int i = 1; i < 30; ++i) { t *= -x * x / ((2 * i) * (2 * i + 1)); s += t; }
    return s;
}
constexpr double taylor_cos(double x) {
    double t = 1, s = 1;
    for (int i = 1; i < 30; ++i) { t *= -x * x / ((2 * i - 1) * (2 * i)); s += t; }
    return s;
}
// cos and sin of 2 pi k / R: octant reduction to [0, pi/4) and Taylor series;
// exact on the axes.
constexpr CS cos_sin_2pi(int k, int R) {
    k = ((k % R) + R) % R;
    const long long k8 = 8LL * k;
    const int oct = (int)(k8 / R);
    const long long rem = k8 - (long long)oct * R;
    const double x = (kPiD / 4) * (double)rem / (double)R;
    double sx = taylor_sin(x), cx = taylor_cos(x);
    if (rem == 0) { sx = 0; cx = 1; }
    const double r2 = 0.70710678118654752440084436210484903928;
    switch (oct) {
        case 0: return CS{cx, sx};
        case 1: return CS{r2 * (cx - sx), r2 * (cx + sx)};
        case 2: return CS{-sx, cx};
        case 3: return CS{-r2 * (cx + sx), r2 * (cx - sx)};
        case 4: return CS{-cx, -sx};
        case 5: return CS{-r2 * (cx - sx), -r2 * (cx + sx)};
        case 6: return CS{sx, -cx};
        default: return CS{r2 * (cx + sx), -r2 * (cx - sx)};
    }
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
constexpr int bitrev(int i, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}

// One radix-2 butterfly of a length-LEN stage with twiddle W_LEN^K
// (exp(-2 pi i K/LEN) forward, conjugate inverse); trivial twiddles cost no
// multiplication.  Others take six fused multiply-adds: x' = x + w y as two
// chained FMAs per component, then y' = 2 x - x' (which differs from x - w y
// only by the rounding of x').
template <typename T, bool INV, int LEN, int K>
__host__ __device__ __forceinline__ void bfly(cpx<T>& x, cpx<T>& y) {
    if constexpr (K == 0 || 4 * K == LEN) {
        const cpx<T> t = K == 0 ? y : rot90<T, INV>(y);
        y = x - t;
        x = x + t;
    } else {
        constexpr CS w = cos_sin_2pi(K, LEN);
        const T wr = (T)w.c, wi = INV ? (T)w.s : (T)-w.s;
        const T xr = (T)fma(wr, y.x, (T)fma(-wi, y.y, x.x));
        const T xi = (T)fma(wr, y.y, (T)fma(wi, y.x, x.y));
        y = make_cpx<T>((T)fma((T)2, x.x, -xr), (T)fma((T)2, x.y, -xi));
        x = make_cpx<T>(xr, xi);
    }
}

template <typename T, bool INV, int LEN, int... I>
__host__ __device__ __forceinline__ void dft_stage(cpx<T>* a, std::integer_sequence<int, I...>) {
    (bfly<T, INV, LEN, I % (LEN / 2)>(a[(I / (LEN / 2)) * LEN + I % (LEN / 2)],
                                      a[(I / (LEN / 2)) * LEN + I % (LEN / 2) + LEN / 2]),
     ...);
}

template <typename T, bool INV, int R, int LEN>
__host__ __device__ __forceinline__ void dft_stages(cpx<T>* a) {
    if constexpr (LEN <= R) {
        dft_stage<T, INV, LEN>(a, std::make_integer_sequence<int, R / 2>{});
        dft_stages<T, INV, R, LEN * 2>(a);
    }
}

template <typename T, int R, int... I>
__host__ __device__ __forceinline__ void bitrev_copy(cpx<T>* out, const cpx<T>* in,
                                           std::integer_sequence<int, I...>) {
    ((out[I] = in[bitrev(I, ilog2c(R))]), ...);
}

// In-register DFT of length R (power of two), natural order in and out:
// a[k] <- sum_j a[j] exp(-+2 pi i j k / R).  Unnormalised.
template <typename T, int R, bool INV>
__host__ __device__ __forceinline__ void dft_reg(cpx<T> (&a)[R]) {
    if constexpr (R > 1) {
        cpx<T> b[R];
        bitrev_copy<T, R>(b, a, std::make_integer_sequence<int, R>{});
        dft_stages<T, INV, R, 2>(b);
#pragma unroll
        for (int i = 0; i < R; ++i) a[i] = b[i];
    }
}

}  // namespace amap

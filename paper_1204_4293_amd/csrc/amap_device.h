// Device-side building blocks shared by the kernels of the library:
// a small complex type, the Philox4x64-10 counter-based generator, and the
// periodic-index helpers.  Written for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amap {

constexpr int kMaxLogN = 12;          // largest map side 4096
constexpr int kMaxN = 1 << kMaxLogN;

template <typename T>
struct cpx {
    T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cpx<T> make_cpx(T a, T b) { cpx<T> r; r.x = a; r.y = b; return r; }

// Streaming stores for outputs that the next kernel reads back from memory:
// marked non-temporal, so they do not displace cached inputs and leave no
// dirty lines in L2 for the consumer to contend with.
__device__ __forceinline__ void store_stream(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(cpx<float>* p, const cpx<float>& v) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<f2*>(p));
}
__device__ __forceinline__ void store_stream(cpx<double>* p, const cpx<double>& v) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<d2*>(p));
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return make_cpx(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return make_cpx(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return make_cpx(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by the conjugate of b
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
    return make_cpx(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__host__ __device__ __forceinline__ cpx<T> rot90(cpx<T> a) {
    return INV ? make_cpx(-a.y, a.x) : make_cpx(a.y, -a.x);
}

// Sub-grid order of an n x n plane for d = 2^logd: pixel (x, y) belongs to
// sub-grid (p, q) = (x mod d, y mod d), an m x m periodic map (m = n / d) at
// (x', y') = (x / d, y / d); the plane holds the d^2 sub-grids one after the
// other, sub-grid (p, q) at (q d + p) m^2, row-major inside.  idx is the
// row-major index y n + x.
__host__ __device__ __forceinline__ long long subgrid_index(long long idx, int logn, int logd) {
    const int logm = logn - logd;
    const long long x = idx & ((1ll << logn) - 1), y = idx >> logn;
    const long long dm = (1ll << logd) - 1;
    return ((((y & dm) << logd) | (x & dm)) << (2 * logm)) | ((y >> logd) << logm) | (x >> logd);
}

// ---- Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11) ----------------
struct u64x4 { uint64_t v[4]; };

// The 128-bit product of a and b from four 32 x 32 -> 64-bit products, each
// with the carry of the previous ones folded in as a 32-bit addend (no
// partial sum exceeds 64 bits), so the high and low halves share them.
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t p01 = (uint64_t)a0 * b1 + (p00 >> 32);
    const uint64_t p10 = (uint64_t)a1 * b0 + (uint32_t)p01;
    hi = (uint64_t)a1 * b1 + (p01 >> 32) + (p10 >> 32);
    lo = (p10 << 32) | (uint32_t)p00;
}

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                               uint64_t c3, uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, hi0, lo0);
        mulhilo64(M1, c2, hi1, lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    u64x4 r;
    r.v[0] = c0; r.v[1] = c1; r.v[2] = c2; r.v[3] = c3;
    return r;
}

// The eight 32-bit values of block b (pixels 8b .. 8b+7) of realisation r.
__device__ __forceinline__ void philox_block_u32(uint64_t seed, uint64_t r, uint64_t b,
                                                 uint32_t out[8]) {
    const u64x4 w = philox4x64_10(b, r, 0, 0, seed, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        out[2 * i] = (uint32_t)(w.v[i] & 0xFFFFFFFFull);
        out[2 * i + 1] = (uint32_t)(w.v[i] >> 32);
    }
}

// sin and cos of 2 pi w / 2^24 for a 24-bit integer w, single precision:
// w / 2^24 is exact in float and is the angle in turns, the unit of the
// hardware sine and cosine instructions.  Over all 2^24 inputs their
// results are within 1.3e-7 of the true values (checked exhaustively on
// gfx950 against double precision).
__device__ __forceinline__ void sincos_turn24(uint32_t w, float& sn, float& cs) {
    const float t = (float)w * (1.0f / 16777216.0f);
    sn = __builtin_amdgcn_sinf(t);
    cs = __builtin_amdgcn_cosf(t);
}

// Rotation of a shear value by beta = 2 pi u, u = (v >> 8) 2^-24.
__device__ __forceinline__ void rotate_by_u32(uint32_t v, float& a, float& b) {
    float s, c;
    sincos_turn24(v >> 8, s, c);
    const float na = a * c - b * s;
    const float nb = a * s + b * c;
    a = na; b = nb;
}
__device__ __forceinline__ void rotate_by_u32(uint32_t v, double& a, double& b) {
    const double u2 = (double)(v >> 8) * (1.0 / 8388608.0);
    double s, c;
    sincospi(u2, &s, &c);
    const double na = a * c - b * s;
    const double nb = a * s + b * c;
    a = na; b = nb;
}

}  // namespace amap

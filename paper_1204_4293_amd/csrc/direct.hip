// Brute-force aperture mass from the tangential shear (eq:shearmap), the
// comparison method whose O(n^2 cut^2) cost the starlet removes (Sec. 5.1).
//
// M(x) = -sum_d [ Q(|d|) cos2phi_d g1(x+d) + Q(|d|) sin2phi_d g2(x+d) ]
// over the integer offsets 0 < |d|^2 <= cut^2.  The host tabulates the two
// weights per offset; for each row dy of the disc the dx range is contiguous.
//
// Maps from 512 px wide: a workgroup of TH wavefronts computes TH output
// rows of 512 pixels, one row per wavefront and eight consecutive outputs
// per lane.  The input rows the tile needs (y0 - R .. y0 + TH - 1 + R,
// 512 + 2 R4 + 8 columns wide) pass through a ring of RING rows in LDS,
// shared by the TH wavefronts.  Each wavefront walks the taps of its row
// offset dy in groups of four dx: per group it reads one new 4-vector of g1
// and of g2 from LDS, takes the eight weights of the group from the scalar
// cache (dy is uniform across the wavefront) and does 64 fused
// multiply-adds.  Taps outside the disc carry zero weight (the table is
// padded to whole groups).  Smaller maps use the plain kernel below, where
// each thread slides a four-wide window along dx through global memory.
#include "amap_device.h"
#include "amap_launch.h"

namespace amap {

template <typename T>
__global__ void __launch_bounds__(256)
k_map_direct(const T* __restrict__ g1, const T* __restrict__ g2, int logn, int R,
             const int* __restrict__ half, const T* __restrict__ wc, const T* __restrict__ ws,
             T* __restrict__ out) {
    const int n = 1 << logn, m = n - 1;
    const long long n2 = (long long)n * n;
    const long long p0 = ((long long)blockIdx.x * 256 + threadIdx.x) * 4;
    if (p0 >= n2) return;
    const int x = (int)(p0 & m);
    const int y = (int)(p0 >> logn);
    const int D = 2 * R + 1;
    T acc[4] = {(T)0, (T)0, (T)0, (T)0};
    for (int dy = -R; dy <= R; ++dy) {
        const int h = half[dy + R];
        if (h < 0) continue;
        const long long row = (long long)((y + dy) & m) * n;
        const T* wcr = wc + (long long)(dy + R) * D + R;
        const T* wsr = ws + (long long)(dy + R) * D + R;
        T a1[4], a2[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a1[i] = g1[row + ((x - h + i) & m)];
            a2[i] = g2[row + ((x - h + i) & m)];
        }
        for (int dx = -h; dx <= h; ++dx) {
            const T qc = wcr[dx], qs = wsr[dx];
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = fma(qc, a1[i], fma(qs, a2[i], acc[i]));
#pragma unroll
            for (int i = 0; i < 3; ++i) { a1[i] = a1[i + 1]; a2[i] = a2[i + 1]; }
            a1[3] = g1[row + ((x + dx + 4) & m)];
            a2[3] = g2[row + ((x + dx + 4) & m)];
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) out[p0 + i] = -acc[i];
}

// Group table of the LDS kernel: row dy + R holds, for each group of four
// dx starting at dx = 4 k - R4 (k = 0 .. R4 / 2), the four weights Q cos 2phi
// then the four Q sin 2phi (zero outside the disc).
constexpr int kDirectTW = 512;   // outputs per wavefront row
constexpr int kDirectTH = 4;     // rows (wavefronts) per workgroup
constexpr int kDirectRing = 8;   // staged input rows
constexpr size_t kDirectMaxLds = 128 * 1024;

template <typename T>
struct Vec4 { T e[4]; };
template <typename T>
__device__ __forceinline__ Vec4<T> lds_ld4(const T* p) {
    if constexpr (sizeof(T) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 v = *reinterpret_cast<const f4*>(p);
        return Vec4<T>{{v[0], v[1], v[2], v[3]}};
    } else {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 a = *reinterpret_cast<const d2*>(p), b = *reinterpret_cast<const d2*>(p + 2);
        return Vec4<T>{{a[0], a[1], b[0], b[1]}};
    }
}

// The 4 x P taps of one group: dx = dx0 + q (q < 4) for outputs i < P,
// from the window (v0 | v1 | v2) of g1 and (u0 | u1 | u2) of g2 starting at
// dx0; w holds the group's four Q cos 2phi and four Q sin 2phi.
template <typename T, int P>
__device__ __forceinline__ void direct_group(T (&acc)[P], const T* __restrict__ w, const Vec4<T>& v0,
                                             const Vec4<T>& v1, const Vec4<T>& v2, const Vec4<T>& u0,
                                             const Vec4<T>& u1, const Vec4<T>& u2) {
    T v[12], u[12];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = v0.e[j]; v[4 + j] = v1.e[j]; v[8 + j] = v2.e[j];
        u[j] = u0.e[j]; u[4 + j] = u1.e[j]; u[8 + j] = u2.e[j];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const T wc = w[q], ws = w[4 + q];
#pragma unroll
        for (int i = 0; i < P; ++i) acc[i] = fma(wc, v[i + q], fma(ws, u[i + q], acc[i]));
    }
}

template <typename T>
__global__ void __launch_bounds__(64 * kDirectTH)
k_map_direct_rows(const T* __restrict__ g1, const T* __restrict__ g2, int logn, int R, int R4,
                  const int* __restrict__ half, const T* __restrict__ gtab, T* __restrict__ out) {
    constexpr int P = 8, TW = kDirectTW, TH = kDirectTH, RING = kDirectRing, NT = 64 * TH;
    extern __shared__ __align__(16) unsigned char direct_smem[];
    T* ring = reinterpret_cast<T*>(direct_smem);
    const int n = 1 << logn, m = n - 1;
    const int SW = TW + 2 * R4 + 8;                  // staged row width, a multiple of 4
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int ntx = n / TW;
    const int x0 = (blockIdx.x % ntx) * TW, y0 = (blockIdx.x / ntx) * TH;
    const int nrows = TH + 2 * R;                     // input rows y0 - R + k
    const int ng = R4 / 2 + 1;                        // groups per table row
    const int vec_row = SW / 4;                       // 4-vectors per staged row and array
    T acc[P];
#pragma unroll
    for (int i = 0; i < P; ++i) acc[i] = (T)0;
    for (int k0 = 0; k0 < nrows; k0 += RING) {
        const int kn = nrows - k0 < RING ? nrows - k0 : RING;
        __syncthreads();  // every wavefront is done with the ring
        for (int e = threadIdx.x; e < kn * 2 * vec_row; e += NT) {
            const int rr = e / (2 * vec_row), rem = e - rr * 2 * vec_row;
            const int arr = rem >= vec_row, c = rem - arr * vec_row;
            const long long row = (long long)((y0 - R + k0 + rr) & m) * n;
            const T* src = (arr ? g2 : g1) + row + ((x0 - R4 + 4 * c) & m);
            T* dst = ring + (rr * 2 + arr) * SW + 4 * c;
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = src[q];
        }
        __syncthreads();
        for (int kk = 0; kk < kn; ++kk) {
            const int dy = k0 + kk - R - wave;            // uniform across the wavefront
            if (dy < -R || dy > R) continue;
            const int h = half[dy + R];
            if (h < 0) continue;
            const T* r1 = ring + (kk * 2) * SW + 8 * lane + R4;
            const T* r2 = r1 + SW;
            const T* wrow = gtab + (long long)(dy + R) * ng * 8;
            const int gb = -((h + 3) >> 2), ge = h >> 2;   // groups dx0 = 4 g cover [-h, h]
            // the window of group g is the 4-vectors at 4 g, 4 g + 4, 4 g + 8;
            // three groups per iteration, the vectors renamed instead of moved
            Vec4<T> a0 = lds_ld4(r1 + 4 * gb), a1 = lds_ld4(r1 + 4 * gb + 4);
            Vec4<T> c0 = lds_ld4(r2 + 4 * gb), c1 = lds_ld4(r2 + 4 * gb + 4);
            int g = gb;
            for (; g + 2 <= ge; g += 3) {
                const Vec4<T> a2 = lds_ld4(r1 + 4 * g + 8), c2 = lds_ld4(r2 + 4 * g + 8);
                direct_group<T, P>(acc, wrow + (g + R4 / 4) * 8, a0, a1, a2, c0, c1, c2);
                a0 = lds_ld4(r1 + 4 * g + 12);
                c0 = lds_ld4(r2 + 4 * g + 12);
                direct_group<T, P>(acc, wrow + (g + 1 + R4 / 4) * 8, a1, a2, a0, c1, c2, c0);
                a1 = lds_ld4(r1 + 4 * g + 16);
                c1 = lds_ld4(r2 + 4 * g + 16);
                direct_group<T, P>(acc, wrow + (g + 2 + R4 / 4) * 8, a2, a0, a1, c2, c0, c1);
            }
            for (; g <= ge; ++g) {
                const Vec4<T> a2 = lds_ld4(r1 + 4 * g + 8), c2 = lds_ld4(r2 + 4 * g + 8);
                direct_group<T, P>(acc, wrow + (g + R4 / 4) * 8, a0, a1, a2, c0, c1, c2);
                a0 = a1; a1 = a2; c0 = c1; c1 = c2;
            }
        }
    }
    T* o = out + (long long)(y0 + wave) * n + x0 + 8 * lane;
#pragma unroll
    for (int i = 0; i < P; ++i) o[i] = -acc[i];
}

// LDS bytes of the row kernel for an R4-padded cut.
template <typename T>
size_t map_direct_rows_lds(int R4) {
    return (size_t)kDirectRing * 2 * (kDirectTW + 2 * R4 + 8) * sizeof(T);
}

template <typename T>
hipError_t launch_map_direct(int logn, const T* g1, const T* g2, int R, const int* half,
                             const T* wc, const T* ws, const T* gtab, T* out, hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    const int n = 1 << logn;
    const int R4 = (R + 3) / 4 * 4;
    const size_t lds = map_direct_rows_lds<T>(R4);
    if (gtab && n >= kDirectTW && lds <= kDirectMaxLds) {
        static bool attr_set = false;
        if (!attr_set) {
            const hipError_t e = hipFuncSetAttribute((const void*)k_map_direct_rows<T>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)kDirectMaxLds);
            if (e != hipSuccess) return e;
            attr_set = true;
        }
        const unsigned blocks = (unsigned)((n / kDirectTW) * (n / kDirectTH));
        AMAP_LAUNCH("map_direct", s,
                    k_map_direct_rows<T><<<blocks, 64 * kDirectTH, lds, s>>>(g1, g2, logn, R, R4, half,
                                                                            gtab, out));
        return hipGetLastError();
    }
    const unsigned blocks = (unsigned)((n2 / 4 + 255) / 256);
    AMAP_LAUNCH("map_direct", s,
                k_map_direct<T><<<blocks, 256, 0, s>>>(g1, g2, logn, R, half, wc, ws, out));
    return hipGetLastError();
}

// Whether the row kernel runs for this size (the host then builds its
// group table).
bool map_direct_uses_groups(int logn, int R, size_t elem) {
    const int R4 = (R + 3) / 4 * 4;
    const size_t lds = (size_t)kDirectRing * 2 * (kDirectTW + 2 * R4 + 8) * elem;
    return (1 << logn) >= kDirectTW && lds <= kDirectMaxLds;
}

template hipError_t launch_map_direct<float>(int, const float*, const float*, int, const int*,
                                             const float*, const float*, const float*, float*,
                                             hipStream_t);
template hipError_t launch_map_direct<double>(int, const double*, const double*, int, const int*,
                                              const double*, const double*, const double*, double*,
                                              hipStream_t);

}  // namespace amap

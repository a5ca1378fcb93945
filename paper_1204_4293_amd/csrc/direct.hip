// Brute-force aperture mass from the tangential shear (eq:shearmap), the
// comparison method whose O(n^2 cut^2) cost the starlet removes (Sec. 5.1).
//
// M(x) = -sum_d [ Q(|d|) cos2phi_d g1(x+d) + Q(|d|) sin2phi_d g2(x+d) ]
// over the integer offsets 0 < |d|^2 <= cut^2.  The host tabulates the two
// weights per offset; for each row dy of the disc the dx range is contiguous.
// Each thread computes four consecutive outputs of a row and slides a
// four-wide register window along dx, so a tap costs two loads and eight
// fused multiply-adds.  Weights are uniform across the wavefront.
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

template <typename T>
hipError_t launch_map_direct(int logn, const T* g1, const T* g2, int R, const int* half,
                             const T* wc, const T* ws, T* out, hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    const unsigned blocks = (unsigned)((n2 / 4 + 255) / 256);
    AMAP_LAUNCH("map_direct", s,
                k_map_direct<T><<<blocks, 256, 0, s>>>(g1, g2, logn, R, half, wc, ws, out));
    return hipGetLastError();
}

template hipError_t launch_map_direct<float>(int, const float*, const float*, int, const int*,
                                             const float*, const float*, float*, hipStream_t);
template hipError_t launch_map_direct<double>(int, const double*, const double*, int, const int*,
                                              const double*, const double*, double*, hipStream_t);

}  // namespace amap

// Noise statistics, S/N and peak counts (Sec. 1: sigma from the variance of
// randomised reconstructions, S = M_ap / sigma; Sec. 2.2: peak counts), and
// the Philox phase stream behind the randomisation.
#include "amap_device.h"
#include "amap_launch.h"

namespace amap {

template <typename T>
__global__ void __launch_bounds__(256)
k_noise_finalize(const double* __restrict__ M2, int R, int J, long long n2,
                 const T* __restrict__ planes_signal, T* __restrict__ sigma, T* __restrict__ snr) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n2) return;
    for (int j = 0; j < J - 1; ++j) {
        const long long e = (long long)j * n2 + idx;
        double var = M2[e] / (double)(R - 1);
        var = var > 0.0 ? var : 0.0;
        const T sg = (T)sqrt(var);
        sigma[e] = sg;
        if (snr) snr[e] = sg > (T)0 ? planes_signal[e] / sg : (T)0;
    }
}

__global__ void k_zero_f64(double* p, long long count) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = 0.0;
}
__global__ void k_zero_i64(long long* p, long long count) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = 0;
}

// Strict 8-neighbour maxima above thr, periodic.  grid (n*n/256, nplanes).
// One atomic add per wavefront of the ballot's population count.
template <typename T>
__global__ void __launch_bounds__(256)
k_count_peaks(const T* __restrict__ snr, int logn, double thr, long long* __restrict__ counts) {
    const int n = 1 << logn, m = n - 1;
    const long long n2 = (long long)n * n;
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    bool peak = false;
    if (idx < n2) {
        const T* p = snr + (long long)blockIdx.y * n2;
        const int x = (int)(idx & m), y = (int)(idx >> logn);
        const T v = p[idx];
        peak = (double)v > thr;
        if (peak) {
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const long long row = (long long)((y + dy) & m) * n;
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dy == 0 && dx == 0) continue;
                    peak = peak && (v > p[row + ((x + dx) & m)]);
                }
            }
        }
    }
    const unsigned long long mask = __ballot(peak);
    if ((threadIdx.x & 63) == 0 && mask)
        atomicAdd((unsigned long long*)&counts[blockIdx.y], (unsigned long long)__popcll(mask));
}

// Thread t writes the eight 32-bit values of Philox block t.
__global__ void __launch_bounds__(256)
k_phase_u32(int logn, uint64_t seed, uint64_t r, uint32_t* __restrict__ out) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long n2 = 1ll << (2 * logn);
    if (8 * t >= n2) return;
    uint32_t u[8];
    philox_block_u32(seed, r, (uint64_t)t, u);
#pragma unroll
    for (int i = 0; i < 8; ++i) out[8 * t + i] = u[i];
}

static unsigned blocks_for(long long count) { return (unsigned)((count + 255) / 256); }

template <typename T>
hipError_t launch_noise_finalize(int logn, int J, int R, const double* M2,
                                 const T* planes_signal, T* sigma, T* snr, hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    AMAP_LAUNCH("noise_finalize", s,
                k_noise_finalize<T><<<blocks_for(n2), 256, 0, s>>>(M2, R, J, n2, planes_signal,
                                                                   sigma, snr));
    return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, long long count, hipStream_t s) {
    if (count > 0) AMAP_LAUNCH("zero", s, k_zero_f64<<<blocks_for(count), 256, 0, s>>>(p, count));
    return hipGetLastError();
}
hipError_t launch_zero_i64(long long* p, long long count, hipStream_t s) {
    if (count > 0) AMAP_LAUNCH("zero", s, k_zero_i64<<<blocks_for(count), 256, 0, s>>>(p, count));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_count_peaks(int logn, int nplanes, const T* snr, double thr, long long* counts,
                              hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    hipError_t e = launch_zero_i64(counts, nplanes, s);
    if (e != hipSuccess) return e;
    AMAP_LAUNCH("count_peaks", s,
                k_count_peaks<T><<<dim3(blocks_for(n2), nplanes), 256, 0, s>>>(snr, logn, thr,
                                                                               counts));
    return hipGetLastError();
}

hipError_t launch_phase_u32(int logn, uint64_t seed, uint64_t r, uint32_t* out, hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    AMAP_LAUNCH("phase_u32", s, k_phase_u32<<<blocks_for(n2 / 8), 256, 0, s>>>(logn, seed, r, out));
    return hipGetLastError();
}

template hipError_t launch_noise_finalize<float>(int, int, int, const double*, const float*, float*,
                                                 float*, hipStream_t);
template hipError_t launch_noise_finalize<double>(int, int, int, const double*, const double*,
                                                  double*, double*, hipStream_t);
template hipError_t launch_count_peaks<float>(int, int, const float*, double, long long*, hipStream_t);
template hipError_t launch_count_peaks<double>(int, int, const double*, double, long long*, hipStream_t);

}  // namespace amap

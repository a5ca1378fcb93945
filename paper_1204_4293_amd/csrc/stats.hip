// Noise statistics, S/N and peak counts (Sec. 1: sigma from the variance of
// randomised reconstructions, S = M_ap / sigma; Sec. 2.2: peak counts), and
// the Philox phase stream behind the randomisation.
#include "amap_device.h"
#include "amap_launch.h"

namespace amap {

// Index of pixel idx's statistics for scale j under `lay`: for every stage
// on sub-grids that has started by scale j, the pixel's place in the
// current block (the whole plane, then one sub-grid of the stage before)
// goes to that block's sub-grid order for the stage's d.
__device__ __forceinline__ long long stat_index(long long idx, int logn, int j, const StatLayout& lay) {
    long long s = idx;
    int dprev = 0;
    for (int k = 0; k < lay.count && lay.j0[k] <= j; ++k) {
        const int d = lay.j0[k] - 1, lm = logn - dprev;
        const long long mask = (1ll << (2 * lm)) - 1;
        s = (s & ~mask) | subgrid_index(s & mask, lm, d - dprev);
        dprev = d;
    }
    return s;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_noise_finalize(const double* __restrict__ M2, int R, int J, int logn, StatLayout lay,
                 const T* __restrict__ planes_signal, T* __restrict__ sigma, T* __restrict__ snr) {
    const long long n2 = 1ll << (2 * logn);
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n2) return;
    for (int j = 0; j < J - 1; ++j) {
        const long long e = (long long)j * n2 + idx;
        double var = M2[(long long)j * n2 + stat_index(idx, logn, j + 1, lay)] /
                     (double)(R - 1);
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

// Strict 8-neighbour maxima above thr, periodic.  grid (blocks, nplanes) of
// 1024 threads: each block takes chunks of 4096 pixels of its plane in turn (every thread
// four consecutive pixels of a row, n >= 16, so they share the row) and
// loads a neighbourhood only if one of its pixels is above thr.  The block's
// count gathers in LDS and reaches the plane's counter by one atomic add:
// device-wide adds to one address serialise, so there are few of them.
template <typename T>
__global__ void __launch_bounds__(1024)
k_count_peaks(const T* __restrict__ snr, int logn, double thr, long long* __restrict__ counts) {
    __shared__ unsigned int block_count;
    if (threadIdx.x == 0) block_count = 0u;
    const int n = 1 << logn, m = n - 1;
    const long long n2 = (long long)n * n;
    const T* p = snr + (long long)blockIdx.y * n2;
    unsigned int npk = 0;
    for (long long idx = ((long long)blockIdx.x * 1024 + threadIdx.x) * 4; idx < n2;
         idx += (long long)gridDim.x * 4096) {
        const int x = (int)(idx & m), y = (int)(idx >> logn);
        T r[3][6];  // rows y-1, y, y+1 at columns x-1 .. x+4
#pragma unroll
        for (int i = 0; i < 4; ++i) r[1][1 + i] = p[idx + i];
        bool cand[4], any = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            cand[i] = (double)r[1][1 + i] > thr;
            any = any || cand[i];
        }
        if (!any) continue;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const T* row = p + (long long)((y + dy) & m) * n;
            r[dy + 1][0] = row[(x - 1) & m];
            r[dy + 1][5] = row[(x + 4) & m];
            if (dy != 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) r[dy + 1][1 + i] = row[x + i];
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const T v = r[1][1 + i];
            bool pk = cand[i];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    if (a != 1 || b != 1) pk = pk & (v > r[a][i + b]);
            npk += pk ? 1u : 0u;
        }
    }
    __syncthreads();  // block_count is zeroed
    if (npk) atomicAdd(&block_count, npk);
    __syncthreads();
    if (threadIdx.x == 0 && block_count)
        atomicAdd((unsigned long long*)&counts[blockIdx.y], (unsigned long long)block_count);
}

// Histogram of peak heights (Sec. 2.2): pixels that are strict 8-neighbour
// maxima of sign*value, periodic, binned by h = sign*value into nbins equal
// bins over [lo, lo + nbins*width); the bin is floor((h - lo) / width) in
// double.  grid (blocks, nplanes) of 1024 threads, each block striding over
// its plane a pixel per thread at a time (at most 64 blocks per plane);
// counts gather in LDS and are added to hist once per block and bin.
template <typename T>
__global__ void __launch_bounds__(1024)
k_peak_hist(const T* __restrict__ planes, int logn, int sign, double lo, double width, int nbins,
            long long* __restrict__ hist) {
    extern __shared__ unsigned int bins[];
    for (int b = threadIdx.x; b < nbins; b += 1024) bins[b] = 0u;
    __syncthreads();
    const int n = 1 << logn, m = n - 1;
    const long long n2 = (long long)n * n;
    const T* p = planes + (long long)blockIdx.y * n2;
    for (long long idx = (long long)blockIdx.x * 1024 + threadIdx.x; idx < n2;
         idx += (long long)gridDim.x * 1024) {
        const int x = (int)(idx & m), y = (int)(idx >> logn);
        const T h = sign > 0 ? p[idx] : -p[idx];
        // the eight neighbour loads issue together, then one test
        T q[8];
        int k = 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const long long row = (long long)((y + dy) & m) * n;
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx)
                if (dy != 0 || dx != 0) q[k++] = p[row + ((x + dx) & m)];
        }
        bool peak = true;
#pragma unroll
        for (int i = 0; i < 8; ++i) peak = peak & (h > (sign > 0 ? q[i] : -q[i]));
        if (peak) {
            const double b = floor(((double)h - lo) / width);
            if (b >= 0.0 && b < (double)nbins) atomicAdd(&bins[(int)b], 1u);
        }
    }
    __syncthreads();
    long long* out = hist + (long long)blockIdx.y * nbins;
    for (int b = threadIdx.x; b < nbins; b += 1024)
        if (bins[b]) atomicAdd((unsigned long long*)&out[b], (unsigned long long)bins[b]);
}

// ---- plane moments: deterministic two-pass reductions in double -----------------
// Sum of a block's 256 values (fixed order: wave shuffles, then the waves).
__device__ __forceinline__ double block_sum256(double v, double* sh) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return t;
}

// Pass 1: per-block sums of a plane (grid (nb, nplanes)); pass 2 (mean
// given): per-block sums of (x - mean)^k, k = 2, 3, 4.  part is
// [3][nplanes][nb].
template <typename T, bool CENTRAL>
__global__ void __launch_bounds__(256)
k_moment_part(const T* __restrict__ planes, long long n2, const double* __restrict__ out4,
              double* __restrict__ part) {
    __shared__ double sh[4];
    const int pl = blockIdx.y, nb = gridDim.x;
    const T* p = planes + (long long)pl * n2;
    const double mu = CENTRAL ? out4[4 * pl] : 0.0;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n2; i += (long long)nb * 256) {
        const double d = (double)p[i] - mu;
        if (CENTRAL) {
            const double d2 = d * d;
            s1 += d2;
            s2 += d2 * d;
            s3 += d2 * d2;
        } else {
            s1 += d;
        }
    }
    const long long o = (long long)pl * nb + blockIdx.x;
    const long long stride = (long long)gridDim.y * nb;
    const double t1 = block_sum256(s1, sh);
    if (!CENTRAL) {
        if (threadIdx.x == 0) part[o] = t1;
        return;
    }
    const double t2 = block_sum256(s2, sh);
    const double t3 = block_sum256(s3, sh);
    if (threadIdx.x == 0) {
        part[o] = t1;
        part[stride + o] = t2;
        part[2 * stride + o] = t3;
    }
}

// Folds the nb partials of each plane (one block per plane, fixed order):
// the mean (pass 1) or m2, m3, m4 (pass 2) into out4[4 * plane + ...].
template <bool CENTRAL>
__global__ void __launch_bounds__(256)
k_moment_fold(const double* __restrict__ part, int nb, long long n2, double* __restrict__ out4) {
    __shared__ double sh[4];
    const int pl = blockIdx.x, np = gridDim.x;
    const long long stride = (long long)np * nb;
    const int K = CENTRAL ? 3 : 1;
    for (int k = 0; k < K; ++k) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) v += part[k * stride + (long long)pl * nb + b];
        const double t = block_sum256(v, sh);
        if (threadIdx.x == 0) out4[4 * pl + (CENTRAL ? 1 + k : 0)] = t / (double)n2;
    }
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
// Blocks per plane for the peak histogram: chunks of 1024 pixels, at most 64.
static unsigned hist_blocks(long long n2) {
    const long long chunks = (n2 + 1023) / 1024;
    return (unsigned)(chunks < 64 ? chunks : 64);
}
// Blocks per plane for the peak count: chunks of 4096 pixels, at most 64
// blocks (so at most 64 atomic adds per plane's counter).
static unsigned peak_blocks(long long n2) {
    const long long chunks = (n2 + 4095) / 4096;
    return (unsigned)(chunks < 64 ? chunks : 64);
}

template <typename T>
hipError_t launch_noise_finalize(int logn, int J, int R, const double* M2,
                                 const T* planes_signal, T* sigma, T* snr, hipStream_t s,
                                 const StatLayout& layout) {
    const long long n2 = 1ll << (2 * logn);
    if (layout.count < 0 || layout.count > 16) return hipErrorInvalidValue;
    for (int k = 0; k < layout.count; ++k)  // stage starts inside [1, J), increasing
        if (layout.j0[k] < 1 || layout.j0[k] >= J || (k > 0 && layout.j0[k] <= layout.j0[k - 1]))
            return hipErrorInvalidValue;
    AMAP_LAUNCH("noise_finalize", s,
                k_noise_finalize<T><<<blocks_for(n2), 256, 0, s>>>(M2, R, J, logn, layout,
                                                                   planes_signal, sigma, snr));
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
                k_count_peaks<T><<<dim3(peak_blocks(n2), nplanes), 1024, 0, s>>>(snr, logn, thr, counts));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_peak_hist(int logn, int nplanes, const T* planes, int sign, double lo,
                            double width, int nbins, long long* hist, hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    hipError_t e = launch_zero_i64(hist, (long long)nplanes * nbins, s);
    if (e != hipSuccess) return e;
    AMAP_LAUNCH("peak_hist", s,
                k_peak_hist<T><<<dim3(hist_blocks(n2), nplanes), 1024, nbins * sizeof(unsigned int), s>>>(
                    planes, logn, sign, lo, width, nbins, hist));
    return hipGetLastError();
}

int moment_blocks(int logn) {
    const long long n2 = 1ll << (2 * logn);
    long long nb = n2 / (256 * 8);  // about eight values per thread
    return (int)(nb < 1 ? 1 : (nb > 1024 ? 1024 : nb));
}

template <typename T>
hipError_t launch_plane_moments(int logn, int nplanes, const T* planes, double* part, double* out4,
                                hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    const int nb = moment_blocks(logn);
    AMAP_LAUNCH("moments_mean", s,
                k_moment_part<T, false><<<dim3(nb, nplanes), 256, 0, s>>>(planes, n2, out4, part));
    AMAP_LAUNCH("moments_fold", s, k_moment_fold<false><<<nplanes, 256, 0, s>>>(part, nb, n2, out4));
    AMAP_LAUNCH("moments_central", s,
                k_moment_part<T, true><<<dim3(nb, nplanes), 256, 0, s>>>(planes, n2, out4, part));
    AMAP_LAUNCH("moments_fold", s, k_moment_fold<true><<<nplanes, 256, 0, s>>>(part, nb, n2, out4));
    return hipGetLastError();
}

hipError_t launch_phase_u32(int logn, uint64_t seed, uint64_t r, uint32_t* out, hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    AMAP_LAUNCH("phase_u32", s, k_phase_u32<<<blocks_for(n2 / 8), 256, 0, s>>>(logn, seed, r, out));
    return hipGetLastError();
}

template hipError_t launch_noise_finalize<float>(int, int, int, const double*, const float*, float*,
                                                 float*, hipStream_t, const StatLayout&);
template hipError_t launch_noise_finalize<double>(int, int, int, const double*, const double*,
                                                  double*, double*, hipStream_t, const StatLayout&);
template hipError_t launch_count_peaks<float>(int, int, const float*, double, long long*, hipStream_t);
template hipError_t launch_count_peaks<double>(int, int, const double*, double, long long*, hipStream_t);
template hipError_t launch_peak_hist<float>(int, int, const float*, int, double, double, int, long long*,
                                            hipStream_t);
template hipError_t launch_peak_hist<double>(int, int, const double*, int, double, double, int,
                                             long long*, hipStream_t);
template hipError_t launch_plane_moments<float>(int, int, const float*, double*, double*, hipStream_t);
template hipError_t launch_plane_moments<double>(int, int, const double*, double*, double*, hipStream_t);

}  // namespace amap

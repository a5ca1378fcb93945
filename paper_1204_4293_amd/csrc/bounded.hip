// Fields with edges and of any size: the starlet cascade under periodic,
// mirror or zero boundary rules, and the zero extension and read-back
// around the power-of-two KS inversion.
//
// The a trous cascade is that of Sec. 3 (B3 taps (1,4,6,4,1)/16 at dilation
// 2^(j-1), row pass along x then column pass along y, w_j = c_{j-1} - c_j);
// the paper leaves edges open, so the rule is the caller's: periodic (index
// mod n), mirror (whole-sample symmetric: reflection about the first and
// last samples, period 2(n-1)) or zero outside the field, applied to
// c_{j-1} on each axis at every step.  One thread per output pixel; the
// taps of interior pixels are contiguous rows, so the loads coalesce.
#include <hip/hip_runtime.h>

#include "amap_device.h"
#include "amap_launch.h"

namespace amap {

namespace {

// i mapped into [0, n) by the rule; -1 for a sample outside (zero rule).
__device__ __forceinline__ int bc_index(int i, int n, int mode) {
    if (i >= 0 && i < n) return i;
    if (mode == 0) {
        const int k = i % n;
        return k < 0 ? k + n : k;
    }
    if (mode == 1) {
        const int p = 2 * (n - 1);
        int k = i % p;
        if (k < 0) k += p;
        return k < n ? k : p - k;
    }
    return -1;
}

template <typename T>
__device__ __forceinline__ T b3(T a0, T a1, T a2, T a3, T a4) {
    return (T)0.0625 * (a0 + a4) + (T)0.25 * (a1 + a3) + (T)0.375 * a2;
}

// r[y][x] = sum_t h_t c[y][x + (t-2) d]; grid (ceil(nx/256), ny)
template <typename T>
__global__ void __launch_bounds__(256)
k_bc_row(const T* __restrict__ c, T* __restrict__ r, int nx, int d, int mode) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    const T* row = c + (long long)y * nx;
    T v[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const int i = bc_index(x + (t - 2) * d, nx, mode);
        v[t] = i < 0 ? (T)0 : row[i];
    }
    r[(long long)y * nx + x] = b3(v[0], v[1], v[2], v[3], v[4]);
}

// c_next[y][x] = sum_t h_t r[y + (t-2) d][x], w = c_prev - c_next.  c_prev
// and c_next may be the same array: each thread reads and writes only its
// own pixel of them.  grid (ceil(nx/256), ny)
template <typename T>
__global__ void __launch_bounds__(256)
k_bc_col(const T* __restrict__ r, const T* c_prev, T* __restrict__ w, T* c_next, int ny, int nx,
         int d, int mode) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    T v[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const int i = bc_index(y + (t - 2) * d, ny, mode);
        v[t] = i < 0 ? (T)0 : r[(long long)i * nx + x];
    }
    const long long o = (long long)y * nx + x;
    const T cn = b3(v[0], v[1], v[2], v[3], v[4]);
    const T cp = c_prev[o];
    w[o] = cp - cn;
    c_next[o] = cn;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_pad2(const T* __restrict__ g1, const T* __restrict__ g2, int ny, int nx, int P, T* __restrict__ p1,
       T* __restrict__ p2) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= P) return;
    const bool in = y < ny && x < nx;
    const long long o = (long long)y * P + x, i = (long long)y * nx + x;
    p1[o] = in ? g1[i] : (T)0;
    p2[o] = in ? g2[i] : (T)0;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_crop2(const T* __restrict__ kE_p, const T* __restrict__ kB_p, int P, int nx, T* __restrict__ kE,
        T* __restrict__ kB) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    const long long o = (long long)y * nx + x, i = (long long)y * P + x;
    kE[o] = kE_p[i];
    if (kB) kB[o] = kB_p[i];
}

}  // namespace

template <typename T>
hipError_t launch_starlet_bc(int ny, int nx, int J, int mode, const T* image, T* planes, T* tmp,
                             hipStream_t s) {
    const long long plane = (long long)ny * nx;
    T* coarse = planes + (long long)(J - 1) * plane;
    const dim3 grid((nx + 255) / 256, ny);
    for (int j = 1; j < J; ++j) {
        const int d = 1 << (j - 1);
        const T* c_prev = j == 1 ? image : coarse;
        AMAP_LAUNCH("starlet_bc_row", s, k_bc_row<T><<<grid, 256, 0, s>>>(c_prev, tmp, nx, d, mode));
        AMAP_LAUNCH("starlet_bc_col", s,
                    k_bc_col<T><<<grid, 256, 0, s>>>(tmp, c_prev, planes + (long long)(j - 1) * plane,
                                                     coarse, ny, nx, d, mode));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pad2(const T* g1, const T* g2, int ny, int nx, int P, T* p1, T* p2, hipStream_t s) {
    AMAP_LAUNCH("pad", s, k_pad2<T><<<dim3((P + 255) / 256, P), 256, 0, s>>>(g1, g2, ny, nx, P, p1, p2));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_crop2(const T* kE_p, const T* kB_p, int P, int ny, int nx, T* kE, T* kB,
                        hipStream_t s) {
    AMAP_LAUNCH("crop", s,
                k_crop2<T><<<dim3((nx + 255) / 256, ny), 256, 0, s>>>(kE_p, kB_p, P, nx, kE, kB));
    return hipGetLastError();
}

template hipError_t launch_starlet_bc<float>(int, int, int, int, const float*, float*, float*, hipStream_t);
template hipError_t launch_starlet_bc<double>(int, int, int, int, const double*, double*, double*,
                                              hipStream_t);
template hipError_t launch_pad2<float>(const float*, const float*, int, int, int, float*, float*,
                                       hipStream_t);
template hipError_t launch_pad2<double>(const double*, const double*, int, int, int, double*, double*,
                                        hipStream_t);
template hipError_t launch_crop2<float>(const float*, const float*, int, int, int, float*, float*,
                                        hipStream_t);
template hipError_t launch_crop2<double>(const double*, const double*, int, int, int, double*, double*,
                                         hipStream_t);

}  // namespace amap

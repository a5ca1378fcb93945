// Starlet (a trous, B3-spline) decomposition and reconstruction (Sec. 3 and
// eq:splinewl of the paper).  Step j (1-based) smooths c_{j-1} with the taps
// (1,4,6,4,1)/16 at dilation s = 2^(j-1), first along x then along y, with
// periodic indices, and emits w_j = c_{j-1} - c_j.  The running c lives in
// the last plane of the output stack, so no extra plane is needed.
#include "amap_device.h"
#include "amap_launch.h"

namespace amap {

template <typename T>
__device__ __forceinline__ T b3_combine(T a0, T a1, T a2, T a3, T a4) {
    return ((a0 + a4) + (T)4 * (a1 + a3) + (T)6 * a2) * (T)0.0625;
}

// Row pass: tmp = h_s (x) c along x.  grid (n*n/256, batch)
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
              T* __restrict__ w, T* cnext, long long planes_stride, int logn, int s) {
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
    w[(long long)blockIdx.y * planes_stride + idx] = prev - cj;
    cnext[(long long)blockIdx.y * planes_stride + idx] = cj;
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

template <typename T>
hipError_t launch_starlet(const StarletArgs<T>& a) {
    const long long n2 = 1ll << (2 * a.logn);
    const dim3 grid((unsigned)((n2 + 255) / 256), a.batch);
    T* cnext = a.planes + (long long)(a.J - 1) * n2;
    for (int j = 1; j < a.J; ++j) {
        const int s = 1 << (j - 1);
        const T* cprev = (j == 1) ? a.kappa : cnext;
        const long long cstride = (j == 1) ? a.in_stride : a.planes_stride;
        AMAP_LAUNCH("starlet_row", a.stream,
                    k_starlet_row<T><<<grid, 256, 0, a.stream>>>(cprev, cstride, a.tmp, a.logn, s));
        AMAP_LAUNCH("starlet_col", a.stream,
                    k_starlet_col<T><<<grid, 256, 0, a.stream>>>(
                        a.tmp, cprev, cstride, a.planes + (long long)(j - 1) * n2, cnext,
                        a.planes_stride, a.logn, s));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reconstruct(int logn, int J, const T* planes, T* out, hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    AMAP_LAUNCH("reconstruct", s,
                k_reconstruct<T><<<(unsigned)((n2 + 255) / 256), 256, 0, s>>>(planes, out, logn, J));
    return hipGetLastError();
}

template hipError_t launch_starlet<float>(const StarletArgs<float>&);
template hipError_t launch_starlet<double>(const StarletArgs<double>&);
template hipError_t launch_reconstruct<float>(int, int, const float*, float*, hipStream_t);
template hipError_t launch_reconstruct<double>(int, int, const double*, double*, hipStream_t);

}  // namespace amap

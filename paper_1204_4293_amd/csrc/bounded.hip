// Fields with edges and of any size: the starlet cascade under periodic,
// mirror or zero boundary rules (0, 1, 2), the zero extension and read-back
// around the power-of-two KS inversion, the noise realisations' rotation
// and running statistics (Sec. 1, Sec. 5.1: Welford's update in double,
// then sigma and S/N), and peak counts with neighbours taken through the
// edge rule (Sec. 2.2).
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

// r[y][x] = sum_t h_t c[y][x + (t-2) d]; grid (ceil(nx/256), ny, maps),
// map z at c + z c_stride and r + z r_stride
template <typename T>
__global__ void __launch_bounds__(256)
k_bc_row(const T* __restrict__ c, T* __restrict__ r, int nx, int d, int mode, long long c_stride,
         long long r_stride) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    c += blockIdx.z * c_stride;
    r += blockIdx.z * r_stride;
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
// own pixel of them.  grid (ceil(nx/256), ny, maps); map z's w and c_next
// at + z pl_stride
template <typename T>
__global__ void __launch_bounds__(256)
k_bc_col(const T* __restrict__ r, const T* c_prev, T* __restrict__ w, T* c_next, int ny, int nx,
         int d, int mode, long long r_stride, long long cp_stride, long long pl_stride) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    r += blockIdx.z * r_stride;
    c_prev += blockIdx.z * cp_stride;
    w += blockIdx.z * pl_stride;
    c_next += blockIdx.z * pl_stride;
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

// One smoothing step at dilation d as a tile: kBcTW consecutive columns by
// kBcTH rows of one residue class ry (mod d) of the rows, y = ry + d (M0 + m).
// Taps of the column pass then stay in the class (the edge rule maps each
// tap row on its own, so the tile simply loads the mapped rows), and the
// tile stages kBcTH + 4 rows of kBcTW + 4d columns of c_{j-1} once: the row
// pass runs in LDS on all of them, the column pass on the kBcTH middle rows,
// and w_j = c_{j-1} - c_j and c_j are written (c_j to a buffer apart from
// c_{j-1}, whose halo other tiles still read).  grid (column tiles,
// d * row-tile count, maps); dynamic LDS (kBcTH + 4)(kBcTW + 4d + kBcTW) T,
// under 64 KiB up to dilation bc_max_d.
constexpr int kBcTW = 64, kBcTH = 16;
template <typename T>
constexpr int bc_max_d() { return sizeof(T) == 4 ? 128 : 64; }
template <typename T>
__global__ void __launch_bounds__(256)
k_bc_scale_tile(const T* __restrict__ c_prev, T* __restrict__ w, T* __restrict__ c_next, int ny,
                int nx, int d, int mode, long long cp_stride, long long cn_stride, long long w_stride) {
    extern __shared__ unsigned char lds_raw[];
    T* reg = reinterpret_cast<T*>(lds_raw);            // [kBcTH + 4][RW]
    const int RW = kBcTW + 4 * d;
    T* rr = reg + (kBcTH + 4) * RW;                    // [kBcTH + 4][kBcTW]
    const int x0 = blockIdx.x * kBcTW;
    const int ry = blockIdx.y % d, M0 = (blockIdx.y / d) * kBcTH;
    c_prev += blockIdx.z * cp_stride;
    c_next += blockIdx.z * cn_stride;
    w += blockIdx.z * w_stride;
    // stage: region row m is c_{j-1} row bc(ry + d (M0 + m - 2)), region
    // column i is column bc(x0 - 2d + i)
    for (int e = threadIdx.x; e < (kBcTH + 4) * RW; e += 256) {
        const int m = e / RW, i = e - m * RW;
        const int yy = bc_index(ry + d * (M0 + m - 2), ny, mode);
        const int xx = bc_index(x0 - 2 * d + i, nx, mode);
        reg[e] = (yy < 0 || xx < 0) ? (T)0 : c_prev[(long long)yy * nx + xx];
    }
    __syncthreads();
    // row pass on every staged row
    for (int e = threadIdx.x; e < (kBcTH + 4) * kBcTW; e += 256) {
        const int m = e / kBcTW, i = e - m * kBcTW;
        const T* g = reg + m * RW + i;
        rr[e] = b3(g[0], g[d], g[2 * d], g[3 * d], g[4 * d]);
    }
    __syncthreads();
    // column pass on the middle rows
    for (int e = threadIdx.x; e < kBcTH * kBcTW; e += 256) {
        const int m = e / kBcTW, i = e - m * kBcTW;
        const int y = ry + d * (M0 + m), x = x0 + i;
        if (y >= ny || x >= nx) continue;
        const T* g = rr + m * kBcTW + i;
        const T cn = b3(g[0], g[kBcTW], g[2 * kBcTW], g[3 * kBcTW], g[4 * kBcTW]);
        const T cp = reg[(m + 2) * RW + 2 * d + i];
        const long long o = (long long)y * nx + x;
        w[o] = cp - cn;
        c_next[o] = cn;
    }
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

// grid (ceil(nx/256), ny, maps): map z of P x P arrays at + z in_stride,
// of the ny x nx outputs at + z out_stride
template <typename T>
__global__ void __launch_bounds__(256)
k_crop2(const T* __restrict__ kE_p, const T* __restrict__ kB_p, int P, int nx, T* __restrict__ kE,
        T* __restrict__ kB, long long in_stride, long long out_stride) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    const long long o = blockIdx.z * out_stride + (long long)y * nx + x;
    const long long i = blockIdx.z * in_stride + (long long)y * P + x;
    kE[o] = kE_p[i];
    if (kB) kB[o] = kB_p[i];
}

// One Philox block (8 flat pixels) per thread: rotate the shears by the
// phases of realisation r0 + blockIdx.y and scatter them into that
// realisation's P x P arrays (at + blockIdx.y p_stride).
template <typename T>
__global__ void __launch_bounds__(256)
k_rotate_scatter(const T* __restrict__ g1, const T* __restrict__ g2, int ny, int nx, int P,
                 uint64_t seed, uint64_t r0, T* __restrict__ p1, T* __restrict__ p2, long long p_stride) {
    const long long npix = (long long)ny * nx;
    const long long b = (long long)blockIdx.x * 256 + threadIdx.x;
    if (8 * b >= npix) return;
    p1 += blockIdx.y * p_stride;
    p2 += blockIdx.y * p_stride;
    uint32_t u[8];
    philox_block_u32(seed, r0 + blockIdx.y, (uint64_t)b, u);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const long long pix = 8 * b + i;
        if (pix >= npix) break;
        const int y = (int)(pix / nx), x = (int)(pix - (long long)y * nx);
        T a = g1[pix], c = g2[pix];
        rotate_by_u32(u[i], a, c);
        p1[(long long)y * P + x] = a;
        p2[(long long)y * P + x] = c;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_zero2(T* __restrict__ p1, T* __restrict__ p2, long long count) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    p1[i] = (T)0;
    p2[i] = (T)0;
}

// Welford's update with realisations r0 .. r0+nb-1 in order, the b-th's
// values at w + b w_stride (realisation 0 writes M and M2 unread).
template <typename T>
__global__ void __launch_bounds__(256)
k_welford_bc(const T* __restrict__ w, long long w_stride, int nb, double* __restrict__ M,
             double* __restrict__ M2, long long count, int r0) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    double m = r0 == 0 ? 0.0 : M[i], m2 = r0 == 0 ? 0.0 : M2[i];
    for (int b = 0; b < nb; ++b) {
        const double v = (double)w[b * w_stride + i];
        const int r = r0 + b;
        if (r == 0) {
            m = v;
            m2 = 0.0;
            continue;
        }
        const double d = v - m, mn = m + d / (double)(r + 1);
        m2 = m2 + d * (v - mn);
        m = mn;
    }
    M[i] = m;
    M2[i] = m2;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_sigma_snr_bc(const double* __restrict__ M2, int R, const T* __restrict__ w_signal, T* __restrict__ sigma,
               T* __restrict__ snr, long long count) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const double sg = sqrt(M2[i] / (double)(R - 1));
    sigma[i] = (T)sg;
    if (snr) snr[i] = sg > 0.0 ? (T)((double)w_signal[i] / sg) : (T)0;
}

// Strict 8-neighbour maxima above thr of ny x nx planes, neighbours taken
// through the edge rule (0 outside under the zero rule); grid (blocks,
// nplanes) of 1024 threads, each block taking rows of its plane in turn,
// its count gathered in LDS and added once.  With a mask (bytes, non-zero
// = observed) a maximum counts only where its pixel and every neighbour
// inside the field are observed.
template <typename T>
__global__ void __launch_bounds__(1024)
k_count_peaks_bc(const T* __restrict__ planes, const unsigned char* __restrict__ mask, int ny,
                 int nx, int mode, double thr, long long* __restrict__ counts) {
    __shared__ unsigned int block_count;
    if (threadIdx.x == 0) block_count = 0u;
    const long long npix = (long long)ny * nx;
    const T* p = planes + (long long)blockIdx.y * npix;
    unsigned int npk = 0;
    for (int y = blockIdx.x; y < ny; y += gridDim.x) {
        for (int x = threadIdx.x; x < nx; x += 1024) {
            const T v = p[(long long)y * nx + x];
            if (!((double)v > thr)) continue;
            bool pk = !mask || mask[(long long)y * nx + x] != 0;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = bc_index(y + dy, ny, mode);
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dy == 0 && dx == 0) continue;
                    const int xx = bc_index(x + dx, nx, mode);
                    const bool in = yy >= 0 && xx >= 0;
                    const T q = in ? p[(long long)yy * nx + xx] : (T)0;
                    pk = pk && (v > q);
                    if (mask && in) pk = pk && mask[(long long)yy * nx + xx] != 0;
                }
            }
            npk += pk ? 1u : 0u;
        }
    }
    __syncthreads();  // block_count is zeroed
    if (npk) atomicAdd(&block_count, npk);
    __syncthreads();
    if (threadIdx.x == 0 && block_count)
        atomicAdd((unsigned long long*)&counts[blockIdx.y], (unsigned long long)block_count);
}

// Shear of a masked field: both components kept where the mask byte is
// non-zero and zeroed where the pixel is missing; four pixels per thread
// (count a multiple of 4, buffers 256-byte aligned), in place allowed.
template <typename T>
__global__ void __launch_bounds__(256)
k_mask_shear(const T* g1, const T* g2, const unsigned char* __restrict__ mask, T* o1, T* o2,
             long long quads) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= quads) return;
    const uchar4 m = reinterpret_cast<const uchar4*>(mask)[i];
    const unsigned char mm[4] = {m.x, m.y, m.z, m.w};
    T a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) { a[k] = g1[4 * i + k]; b[k] = g2[4 * i + k]; }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        o1[4 * i + k] = mm[k] ? a[k] : (T)0;
        o2[4 * i + k] = mm[k] ? b[k] : (T)0;
    }
}

// The last count % 4 pixels.
template <typename T>
__global__ void k_mask_shear_tail(const T* g1, const T* g2, const unsigned char* __restrict__ mask,
                                  T* o1, T* o2, long long first, long long count) {
    const long long i = first + threadIdx.x;
    if (i >= count) return;
    const T a = g1[i], b = g2[i];
    o1[i] = mask[i] ? a : (T)0;
    o2[i] = mask[i] ? b : (T)0;
}

}  // namespace

template <typename T>
hipError_t launch_count_peaks_bc(int ny, int nx, int nplanes, int mode, const T* planes,
                                 const unsigned char* mask, double thr, long long* counts,
                                 hipStream_t s) {
    hipError_t e = launch_zero_i64(counts, nplanes, s);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)(ny < 256 ? ny : 256);  // at most 256 adds per counter
    AMAP_LAUNCH("count_peaks_bc", s,
                k_count_peaks_bc<T><<<dim3(blocks, nplanes), 1024, 0, s>>>(planes, mask, ny, nx, mode,
                                                                          thr, counts));
    return hipGetLastError();
}
template hipError_t launch_count_peaks_bc<float>(int, int, int, int, const float*, const unsigned char*,
                                                 double, long long*, hipStream_t);
template hipError_t launch_count_peaks_bc<double>(int, int, int, int, const double*, const unsigned char*,
                                                  double, long long*, hipStream_t);

template <typename T>
hipError_t launch_mask_shear(long long count, const T* g1, const T* g2, const unsigned char* mask,
                             T* o1, T* o2, hipStream_t s) {
    const long long quads = count / 4;
    if (quads > 0)
        AMAP_LAUNCH("mask_shear", s,
                    k_mask_shear<T><<<(unsigned)((quads + 255) / 256), 256, 0, s>>>(g1, g2, mask, o1, o2,
                                                                                   quads));
    if (count % 4)
        AMAP_LAUNCH("mask_shear", s,
                    k_mask_shear_tail<T><<<1, 4, 0, s>>>(g1, g2, mask, o1, o2, 4 * quads, count));
    return hipGetLastError();
}
template hipError_t launch_mask_shear<float>(long long, const float*, const float*, const unsigned char*,
                                             float*, float*, hipStream_t);
template hipError_t launch_mask_shear<double>(long long, const double*, const double*,
                                              const unsigned char*, double*, double*, hipStream_t);

template <typename T>
hipError_t launch_starlet_bc(int ny, int nx, int J, int mode, const T* image, T* planes, T* tmp,
                             int maps, long long image_stride, long long planes_stride, hipStream_t s) {
    const long long plane = (long long)ny * nx;
    T* coarse = planes + (long long)(J - 1) * plane;
    // scales 1 .. jt (dilation <= bc_max_d) run as tiles, alternating their
    // c_j between tmp and the coarse plane so that c_jt lands in the coarse
    // plane; the later scales run a row and a column pass in place there
    int jt = 0;
    while (jt + 1 < J && (1 << jt) <= bc_max_d<T>()) ++jt;
    const T* c_prev = image;
    long long cp_stride = image_stride;
    for (int j = 1; j <= jt; ++j) {
        const int d = 1 << (j - 1);
        const bool to_coarse = ((jt - j) & 1) == 0;
        T* dst = to_coarse ? coarse : tmp;
        const long long dst_stride = to_coarse ? planes_stride : plane;
        const int rows = (ny + d - 1) / d;  // rows of the largest residue class
        const int row_tiles = (rows + kBcTH - 1) / kBcTH;
        const dim3 grid((nx + kBcTW - 1) / kBcTW, d * row_tiles, maps);
        const size_t lds = (size_t)(kBcTH + 4) * (kBcTW + 4 * d + kBcTW) * sizeof(T);
        AMAP_LAUNCH("starlet_bc_tile", s,
                    k_bc_scale_tile<T><<<grid, 256, lds, s>>>(c_prev, planes + (long long)(j - 1) * plane,
                                                              dst, ny, nx, d, mode, cp_stride, dst_stride,
                                                              planes_stride));
        c_prev = dst;
        cp_stride = dst_stride;
    }
    const dim3 grid((nx + 255) / 256, ny, maps);
    for (int j = jt + 1; j < J; ++j) {
        const int d = 1 << (j - 1);
        AMAP_LAUNCH("starlet_bc_row", s,
                    k_bc_row<T><<<grid, 256, 0, s>>>(c_prev, tmp, nx, d, mode, cp_stride, plane));
        AMAP_LAUNCH("starlet_bc_col", s,
                    k_bc_col<T><<<grid, 256, 0, s>>>(tmp, c_prev, planes + (long long)(j - 1) * plane,
                                                     coarse, ny, nx, d, mode, plane, cp_stride,
                                                     planes_stride));
        c_prev = coarse;
        cp_stride = planes_stride;
    }
    return hipGetLastError();
}
template <typename T>
hipError_t launch_pad2(const T* g1, const T* g2, int ny, int nx, int P, T* p1, T* p2, hipStream_t s) {
    AMAP_LAUNCH("pad", s, k_pad2<T><<<dim3((P + 255) / 256, P), 256, 0, s>>>(g1, g2, ny, nx, P, p1, p2));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_crop2(const T* kE_p, const T* kB_p, int P, int ny, int nx, T* kE, T* kB, int maps,
                        long long in_stride, long long out_stride, hipStream_t s) {
    AMAP_LAUNCH("crop", s,
                k_crop2<T><<<dim3((nx + 255) / 256, ny, maps), 256, 0, s>>>(kE_p, kB_p, P, nx, kE, kB,
                                                                           in_stride, out_stride));
    return hipGetLastError();
}

static unsigned blocks256(long long count) { return (unsigned)((count + 255) / 256); }

template <typename T>
hipError_t launch_rotate_scatter(const T* g1, const T* g2, int ny, int nx, int P, uint64_t seed,
                                 uint64_t r0, int nb, T* p1, T* p2, long long p_stride, hipStream_t s) {
    const long long nblk = ((long long)ny * nx + 7) / 8;
    AMAP_LAUNCH("rotate_scatter", s,
                k_rotate_scatter<T><<<dim3(blocks256(nblk), nb), 256, 0, s>>>(g1, g2, ny, nx, P, seed, r0,
                                                                              p1, p2, p_stride));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zero2(T* p1, T* p2, long long count, hipStream_t s) {
    AMAP_LAUNCH("zero", s, k_zero2<T><<<blocks256(count), 256, 0, s>>>(p1, p2, count));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_welford_bc(const T* w, long long w_stride, int nb, double* M, double* M2,
                             long long count, int r0, hipStream_t s) {
    AMAP_LAUNCH("welford_bc", s,
                k_welford_bc<T><<<blocks256(count), 256, 0, s>>>(w, w_stride, nb, M, M2, count, r0));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sigma_snr_bc(const double* M2, int R, const T* w_signal, T* sigma, T* snr,
                               long long count, hipStream_t s) {
    AMAP_LAUNCH("sigma_snr_bc", s,
                k_sigma_snr_bc<T><<<blocks256(count), 256, 0, s>>>(M2, R, w_signal, sigma, snr, count));
    return hipGetLastError();
}

#define AMAP_BOUNDED_NOISE(T)                                                                            \
    template hipError_t launch_rotate_scatter<T>(const T*, const T*, int, int, int, uint64_t, uint64_t,  \
                                                 int, T*, T*, long long, hipStream_t);                   \
    template hipError_t launch_zero2<T>(T*, T*, long long, hipStream_t);                                 \
    template hipError_t launch_welford_bc<T>(const T*, long long, int, double*, double*, long long, int, \
                                             hipStream_t);                                               \
    template hipError_t launch_sigma_snr_bc<T>(const double*, int, const T*, T*, T*, long long, hipStream_t);
AMAP_BOUNDED_NOISE(float)
AMAP_BOUNDED_NOISE(double)
#undef AMAP_BOUNDED_NOISE

template hipError_t launch_starlet_bc<float>(int, int, int, int, const float*, float*, float*, int,
                                             long long, long long, hipStream_t);
template hipError_t launch_starlet_bc<double>(int, int, int, int, const double*, double*, double*, int,
                                              long long, long long, hipStream_t);
template hipError_t launch_pad2<float>(const float*, const float*, int, int, int, float*, float*,
                                       hipStream_t);
template hipError_t launch_pad2<double>(const double*, const double*, int, int, int, double*, double*,
                                        hipStream_t);
template hipError_t launch_crop2<float>(const float*, const float*, int, int, int, float*, float*, int,
                                        long long, long long, hipStream_t);
template hipError_t launch_crop2<double>(const double*, const double*, int, int, int, double*, double*,
                                         int, long long, long long, hipStream_t);

}  // namespace amap

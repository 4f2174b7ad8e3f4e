// FFT staging of the general SHT on gfx950 (Sect. 3, steps "FFT" and the
// deconvolution / zero-padding part of "NUFFT", and their adjoints).
//
// Layouts
//   D [ncol][nd]      doubled meridians (theta-major inside a column), one column per m
//   E [ncol][n1]      oversampled theta spectrum / theta samples per column
//   G [nrows][n2]     complex torus rows (spin > 0), or half spectrum [nrows][n2/2 + 1]
//                     for the real spin-0 grid
// Column index: spin 0 -> col = m (0..mmax); spin s -> col = m + mmax.
// Kept torus rows: stored row r <-> torus row a = (r + a_min) mod n1.
//
// Deconvolution factor of mode (k, m):  kfac1[|k|] * kfac2[|m|], with
//   kfac1[k] = h1 / (nd psihat1(k)),  kfac2[m] = h2 / psihat2(m),  h = 2 pi / n,
// applied once on the way in (forward) and once on the way out (adjoint), which
// makes the adjoint the exact transpose of the forward.
#include "gsht_internal.hpp"

namespace gsht {

template <typename T> struct cplx2;
template <> struct cplx2<float> { using type = float2; };
template <> struct cplx2<double> { using type = double2; };

template <typename T>
__global__ void zero_kernel(T *__restrict__ p, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = T{};
}

template <typename T>
__global__ void fill_kernel(T *__restrict__ p, T v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_real(void *ptr, double value, int64_t n, int prec, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(fill_kernel<double>, dim3(nb), dim3(256), 0, s, (double *)ptr, value, n);
    else
        hipLaunchKernelGGL(fill_kernel<float>, dim3(nb), dim3(256), 0, s, (float *)ptr,
                           (float)value, n);
    return hipGetLastError();
}

hipError_t launch_zero(void *ptr, size_t bytes, hipStream_t s)
{
    if (bytes == 0)
        return hipSuccess;
    if (bytes % 16 == 0 && ((uintptr_t)ptr % 16) == 0) {
        const size_t n = bytes / 16;
        const unsigned nb = (unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
        hipLaunchKernelGGL(zero_kernel<int4>, dim3(nb), dim3(256), 0, s, (int4 *)ptr, n);
    } else {
        const size_t n = bytes;
        const unsigned nb = (unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
        hipLaunchKernelGGL(zero_kernel<unsigned char>, dim3(nb), dim3(256), 0, s,
                           (unsigned char *)ptr, n);
    }
    return hipGetLastError();
}

__device__ inline int col_to_m(int col, int spin, int mmax) { return spin ? col - mmax : col; }

// Forward: E[col][a] = D^[col][k mod nd] * f(k, m) for |k| <= lmax at a = k mod n1, else 0.
template <typename T>
__global__ void deconv_fwd_kernel(const typename cplx2<T>::type *__restrict__ D,
                                  const double *__restrict__ kf1, const double *__restrict__ kf2,
                                  int lmax, int mmax, int spin, int nd, int n1,
                                  typename cplx2<T>::type *__restrict__ E)
{
    const int col = blockIdx.y;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n1)
        return;
    const int m = col_to_m(col, spin, mmax);
    const int k = (a <= n1 / 2) ? a : a - n1;
    typename cplx2<T>::type v;
    v.x = 0;
    v.y = 0;
    const int ak = k < 0 ? -k : k;
    if (ak <= lmax) {
        const int kd = k < 0 ? k + nd : k;
        const typename cplx2<T>::type d = D[(size_t)col * nd + kd];
        const double f = kf1[ak] * kf2[m < 0 ? -m : m];
        v.x = (T)(f * (double)d.x);
        v.y = (T)(f * (double)d.y);
    }
    E[(size_t)col * n1 + a] = v;
}

// Adjoint: D[col][i] = E^[col][k mod n1] * f(k, m) for i = k mod nd, |k| <= lmax, else 0.
template <typename T>
__global__ void deconv_adj_kernel(const typename cplx2<T>::type *__restrict__ E,
                                  const double *__restrict__ kf1, const double *__restrict__ kf2,
                                  int lmax, int mmax, int spin, int nd, int n1,
                                  typename cplx2<T>::type *__restrict__ D)
{
    const int col = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd)
        return;
    const int m = col_to_m(col, spin, mmax);
    const int k = (i <= nd / 2) ? i : i - nd;
    typename cplx2<T>::type v;
    v.x = 0;
    v.y = 0;
    const int ak = k < 0 ? -k : k;
    if (ak <= lmax) {
        const int ka = k < 0 ? k + n1 : k;
        const typename cplx2<T>::type e = E[(size_t)col * n1 + ka];
        const double f = kf1[ak] * kf2[m < 0 ? -m : m];
        v.x = (T)(f * (double)e.x);
        v.y = (T)(f * (double)e.y);
    }
    D[(size_t)col * nd + i] = v;
}

hipError_t launch_deconv_fwd(const gsht_plan &p, hipStream_t s)
{
    dim3 blk(256), grd((p.n1 + 255) / 256, p.ncol);
    if (p.prec == GSHT_F64)
        hipLaunchKernelGGL(deconv_fwd_kernel<double>, grd, blk, 0, s, (const double2 *)p.D,
                           p.kfac1, p.kfac2, p.lmax, p.mmax, p.spin, p.nd, p.n1, (double2 *)p.E);
    else
        hipLaunchKernelGGL(deconv_fwd_kernel<float>, grd, blk, 0, s, (const float2 *)p.D, p.kfac1,
                           p.kfac2, p.lmax, p.mmax, p.spin, p.nd, p.n1, (float2 *)p.E);
    return hipGetLastError();
}

hipError_t launch_deconv_adj(const gsht_plan &p, hipStream_t s)
{
    dim3 blk(256), grd((p.nd + 255) / 256, p.ncol);
    if (p.prec == GSHT_F64)
        hipLaunchKernelGGL(deconv_adj_kernel<double>, grd, blk, 0, s, (const double2 *)p.E,
                           p.kfac1, p.kfac2, p.lmax, p.mmax, p.spin, p.nd, p.n1, (double2 *)p.D);
    else
        hipLaunchKernelGGL(deconv_adj_kernel<float>, grd, blk, 0, s, (const float2 *)p.E, p.kfac1,
                           p.kfac2, p.lmax, p.mmax, p.spin, p.nd, p.n1, (float2 *)p.D);
    return hipGetLastError();
}

// Tiled transposes through LDS (32 x 32 tiles, 32 x 8 threads).
constexpr int TT = 32;
constexpr int TR = 8;

// Forward: G[r][b] = E[col(b)][(r + a_min) mod n1]  (0 where b has no column).
// gcols = n2 (spin > 0, b -> m = b or b - n2) or n2/2 + 1 (spin 0, m = b).
template <typename T>
__global__ void transpose_fwd_kernel(const typename cplx2<T>::type *__restrict__ E, int mmax,
                                     int spin, int n1, int n2, int gcols, int nrows, int a_min,
                                     typename cplx2<T>::type *__restrict__ G)
{
    __shared__ typename cplx2<T>::type tile[TT][TT + 1];
    const int b0 = blockIdx.x * TT, r0 = blockIdx.y * TT;
    const int tx = threadIdx.x, ty = threadIdx.y;
    // load: rows of the tile are columns b (i.e. E rows), contiguous in r
    for (int yy = ty; yy < TT; yy += TR) {
        const int b = b0 + yy, r = r0 + tx;
        typename cplx2<T>::type v;
        v.x = 0;
        v.y = 0;
        if (b < gcols && r < nrows) {
            int m = spin ? (b <= n2 / 2 ? b : b - n2) : b;
            const int am = m < 0 ? -m : m;
            if (am <= mmax) {
                const int col = spin ? m + mmax : m;
                int a = r + a_min;
                a %= n1;
                if (a < 0)
                    a += n1;
                v = E[(size_t)col * n1 + a];
            }
        }
        tile[yy][tx] = v;
    }
    __syncthreads();
    for (int yy = ty; yy < TT; yy += TR) {
        const int r = r0 + yy, b = b0 + tx;
        if (r < nrows && b < gcols)
            G[(size_t)r * gcols + b] = tile[tx][yy];
    }
}

// Adjoint: E[col][a] = G[(a - a_min) mod n1][b(col)] if that row is kept, else 0
// (with all_rows == 0 the rows that are not kept are left untouched: the fused
// column stage reads kept rows only).
template <typename T>
__global__ void transpose_adj_kernel(const typename cplx2<T>::type *__restrict__ G, int mmax,
                                     int spin, int n1, int n2, int gcols, int nrows, int a_min,
                                     int ncol, int all_rows,
                                     typename cplx2<T>::type *__restrict__ E)
{
    __shared__ typename cplx2<T>::type tile[TT][TT + 1];
    const int c0 = blockIdx.x * TT, a0 = blockIdx.y * TT;
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int yy = ty; yy < TT; yy += TR) {
        const int a = a0 + yy, col = c0 + tx;
        typename cplx2<T>::type v;
        v.x = 0;
        v.y = 0;
        if (a < n1 && col < ncol) {
            int r = (a - a_min) % n1;
            if (r < 0)
                r += n1;
            if (r < nrows) {
                const int m = col_to_m(col, spin, mmax);
                const int b = m < 0 ? m + n2 : m;
                v = G[(size_t)r * gcols + b];
            }
        }
        tile[yy][tx] = v;
    }
    __syncthreads();
    for (int yy = ty; yy < TT; yy += TR) {
        const int col = c0 + yy, a = a0 + tx;
        if (col < ncol && a < n1) {
            if (!all_rows) {
                int r = (a - a_min) % n1;
                if (r < 0)
                    r += n1;
                if (r >= nrows)
                    continue;
            }
            E[(size_t)col * n1 + a] = tile[tx][yy];
        }
    }
}

static int grid_cols(const gsht_plan &p) { return p.spin ? p.n2 : p.n2 / 2 + 1; }

hipError_t launch_transpose_fwd(const gsht_plan &p, hipStream_t s)
{
    const int gc = grid_cols(p);
    dim3 blk(TT, TR), grd((gc + TT - 1) / TT, (p.nrows + TT - 1) / TT);
    if (p.prec == GSHT_F64)
        hipLaunchKernelGGL(transpose_fwd_kernel<double>, grd, blk, 0, s, (const double2 *)p.E,
                           p.mmax, p.spin, p.n1, p.n2, gc, p.nrows, p.a_min,
                           (double2 *)p.G);
    else
        hipLaunchKernelGGL(transpose_fwd_kernel<float>, grd, blk, 0, s, (const float2 *)p.E,
                           p.mmax, p.spin, p.n1, p.n2, gc, p.nrows, p.a_min,
                           (float2 *)p.G);
    return hipGetLastError();
}

hipError_t launch_transpose_adj(const gsht_plan &p, hipStream_t s)
{
    const int gc = grid_cols(p);
    dim3 blk(TT, TR), grd((p.ncol + TT - 1) / TT, (p.n1 + TT - 1) / TT);
    const int all_rows = p.colmode == 2 ? 0 : 1;
    if (p.prec == GSHT_F64)
        hipLaunchKernelGGL(transpose_adj_kernel<double>, grd, blk, 0, s, (const double2 *)p.G,
                           p.mmax, p.spin, p.n1, p.n2, gc, p.nrows, p.a_min, p.ncol, all_rows,
                           (double2 *)p.E);
    else
        hipLaunchKernelGGL(transpose_adj_kernel<float>, grd, blk, 0, s, (const float2 *)p.G,
                           p.mmax, p.spin, p.n1, p.n2, gc, p.nrows, p.a_min, p.ncol, all_rows,
                           (float2 *)p.E);
    return hipGetLastError();
}

}  // namespace gsht

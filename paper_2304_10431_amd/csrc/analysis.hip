// Map analysis on the minimal equiangular ring grid (Appendix A): lmax + 2 rings
// theta_j = pi j / (lmax + 1), both poles included, nphi >= 2 mmax + 1 equidistant
// points per ring.  Along the doubled meridian (north pole -> south pole -> back on
// the opposite side, nd = 2 lmax + 2 samples) a band-limited field is a
// trigonometric polynomial of degree lmax, so it is known everywhere; the
// integral over theta with the weight sin(theta) is then taken exactly in Fourier
// space and folded back onto the original rings, where the adjoint Legendre step
// (the same kernels as the adjoint synthesis) finishes the analysis.
//
// Per column m, with h(theta) the ring values (times the phi quadrature weight):
//   c_k = (1/nd) sum_j h(theta_j) e^{-i k theta_j}                    (|k| <= lmax)
//   h on the twice finer grid theta'_i = 2 pi i / N', N' = 2 nd      (zero padding)
//   v_i = h(theta'_i) u_i,  u_i = (1/N') sum_{|n| <= 2 lmax} W_n e^{-i n theta'_i},
//   W_n = int_0^{2 pi} e^{i n t} |sin t| dt = 4 / (1 - n^2) (n even), 0 (n odd)
//   g_k = sum_i v_i e^{i k theta'_i}                                  (|k| <= lmax)
//   D'_j = (1 / (2 nd)) sum_k g_k e^{-i k theta_j}
// and then a_lm = sum_j lambda_lm(theta_j) D'_j over the doubled meridian, i.e. the
// undoubling and adjoint Legendre steps applied to D'.
#include "gsht_internal.hpp"

namespace gsht {

namespace {

template <typename T> struct cpa;
template <> struct cpa<float> { using type = float2; };
template <> struct cpa<double> { using type = double2; };

// P[j][k] = map[0][j][k] + i map[1][j][k] (spin > 0) or map[0][j][k] (spin 0).
template <typename T>
__global__ void pack_rows_kernel(const T *__restrict__ map, int spin, int64_t n,
                                 typename cpa<T>::type *__restrict__ P)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        typename cpa<T>::type v;
        v.x = map[i];
        v.y = spin ? map[n + i] : (T)0;
        P[i] = v;
    }
}

// Doubled columns from the phi transforms of the rings:
// D[col][j] = scale H_m(theta_j), D[col][nd - j] = (-1)^(s+m) scale H_m(theta_j).
template <typename T>
__global__ void gather_cols_kernel(const typename cpa<T>::type *__restrict__ P, int ntheta,
                                   int nphi, int nd, int mmax, int spin, double scale,
                                   typename cpa<T>::type *__restrict__ D)
{
    const int col = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntheta)
        return;
    const int m = spin ? col - mmax : col;
    const int mi = m >= 0 ? m : m + nphi;
    typename cpa<T>::type v = P[(size_t)j * nphi + mi];
    v.x = (T)(scale * (double)v.x);
    v.y = (T)(scale * (double)v.y);
    typename cpa<T>::type *d = D + (size_t)col * nd;
    d[j] = v;
    if (j > 0 && j < ntheta - 1) {
        const T ms = ((spin + m) & 1) ? (T)-1 : (T)1;
        typename cpa<T>::type w;
        w.x = ms * v.x;
        w.y = ms * v.y;
        d[nd - j] = w;
    }
}

// Up[col][k mod n2] = scale X[col][k mod n1] for |k| <= kmax, 0 elsewhere (n2 > n1).
template <typename T>
__global__ void pad_kernel(const typename cpa<T>::type *__restrict__ X, int n1, int n2, int kmax,
                           double scale, typename cpa<T>::type *__restrict__ Up)
{
    const int col = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2)
        return;
    const int k = i <= n2 / 2 ? i : i - n2;
    typename cpa<T>::type v{};
    if (k >= -kmax && k <= kmax) {
        v = X[(size_t)col * n1 + (k >= 0 ? k : k + n1)];
        v.x = (T)(scale * (double)v.x);
        v.y = (T)(scale * (double)v.y);
    }
    Up[(size_t)col * n2 + i] = v;
}

// X[col][k mod n1] = scale Up[col][k mod n2] for |k| <= kmax, 0 elsewhere (n2 > n1).
template <typename T>
__global__ void trunc_kernel(const typename cpa<T>::type *__restrict__ Up, int n1, int n2,
                             int kmax, double scale, typename cpa<T>::type *__restrict__ X)
{
    const int col = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n1)
        return;
    const int k = i <= n1 / 2 ? i : i - n1;
    typename cpa<T>::type v{};
    if (k >= -kmax && k <= kmax) {
        v = Up[(size_t)col * n2 + (k >= 0 ? k : k + n2)];
        v.x = (T)(scale * (double)v.x);
        v.y = (T)(scale * (double)v.y);
    }
    X[(size_t)col * n1 + i] = v;
}

template <typename T>
__global__ void weight_cols_kernel(typename cpa<T>::type *__restrict__ Up, int n2,
                                   const double *__restrict__ u)
{
    const int col = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2)
        return;
    typename cpa<T>::type v = Up[(size_t)col * n2 + i];
    v.x = (T)(u[i] * (double)v.x);
    v.y = (T)(u[i] * (double)v.y);
    Up[(size_t)col * n2 + i] = v;
}

unsigned eblocks(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

}  // namespace

hipError_t launch_pack_rows(const void *map, int spin, int64_t n, int prec, void *P, hipStream_t s)
{
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(pack_rows_kernel<double>, dim3(eblocks(n)), dim3(256), 0, s,
                           (const double *)map, spin, n, (double2 *)P);
    else
        hipLaunchKernelGGL(pack_rows_kernel<float>, dim3(eblocks(n)), dim3(256), 0, s,
                           (const float *)map, spin, n, (float2 *)P);
    return hipGetLastError();
}

hipError_t launch_gather_cols(const void *P, int ntheta, int nphi, int nd, int mmax, int spin,
                              int ncol, double scale, int prec, void *D, hipStream_t s)
{
    dim3 blk(256), grd((ntheta + 255) / 256, ncol);
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(gather_cols_kernel<double>, grd, blk, 0, s, (const double2 *)P, ntheta,
                           nphi, nd, mmax, spin, scale, (double2 *)D);
    else
        hipLaunchKernelGGL(gather_cols_kernel<float>, grd, blk, 0, s, (const float2 *)P, ntheta,
                           nphi, nd, mmax, spin, scale, (float2 *)D);
    return hipGetLastError();
}

hipError_t launch_pad_cols(const void *X, int n1, int n2, int kmax, int ncol, double scale,
                           int prec, void *Up, hipStream_t s)
{
    dim3 blk(256), grd((n2 + 255) / 256, ncol);
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(pad_kernel<double>, grd, blk, 0, s, (const double2 *)X, n1, n2, kmax,
                           scale, (double2 *)Up);
    else
        hipLaunchKernelGGL(pad_kernel<float>, grd, blk, 0, s, (const float2 *)X, n1, n2, kmax,
                           scale, (float2 *)Up);
    return hipGetLastError();
}

hipError_t launch_trunc_cols(const void *Up, int n1, int n2, int kmax, int ncol, double scale,
                             int prec, void *X, hipStream_t s)
{
    dim3 blk(256), grd((n1 + 255) / 256, ncol);
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(trunc_kernel<double>, grd, blk, 0, s, (const double2 *)Up, n1, n2, kmax,
                           scale, (double2 *)X);
    else
        hipLaunchKernelGGL(trunc_kernel<float>, grd, blk, 0, s, (const float2 *)Up, n1, n2, kmax,
                           scale, (float2 *)X);
    return hipGetLastError();
}

hipError_t launch_weight_cols(void *Up, int n2, int ncol, const double *u, int prec,
                              hipStream_t s)
{
    dim3 blk(256), grd((n2 + 255) / 256, ncol);
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(weight_cols_kernel<double>, grd, blk, 0, s, (double2 *)Up, n2, u);
    else
        hipLaunchKernelGGL(weight_cols_kernel<float>, grd, blk, 0, s, (float2 *)Up, n2, u);
    return hipGetLastError();
}

}  // namespace gsht

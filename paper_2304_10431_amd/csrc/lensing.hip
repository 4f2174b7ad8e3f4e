// Lensing geometry on gfx950 (Sect. 2 and the end of Sect. 3): deflected
// ("unlensed") positions n' from a deflection field, the spin phase chi, the
// coefficient scaling sqrt(l (l + 1)) that turns a lensing potential into the
// gradient-mode coefficients of the spin-1 deflection field, and the
// vector-Jacobian products of these elementwise steps.
//
// Geometry.  At n = (theta, phi) with local basis (e_theta, e_phi) and deflection
// alpha = a_t e_theta + a_p e_phi, |alpha| = a:
//   n' = cos(a) n + (sin(a) / a) (a_t e_theta + a_p e_phi),
// the point at distance a along the great circle.  The spin phase is the angle
// chi by which the basis parallel-transported from n to n' along that great circle
// differs from the local basis at n': with E1 the transport of e_theta,
//   chi = -atan2(E1 . e_phi', E1 . e_theta'),
// which equals the difference beta - beta' of the angles the great circle makes
// with e_theta at its two ends; a spin-s field is lensed as
//   sT_len(n) = e^{i s chi} sT_unl(n').
// The transport is the rotation about k = n x n' that takes n to n'.  Everything
// is written in the frame rotated by -phi about the z axis, where
// n = (sin t, 0, cos t), e_theta = (cos t, 0, -sin t), e_phi = (0, 1, 0).
//
// The same code runs on dual numbers (value and the two partial derivatives with
// respect to (a_t, a_p)), which gives the exact Jacobian for the gradients.
#include "gsht_internal.hpp"

namespace gsht {

namespace {

struct Dual {
    double v, a, b;  // value, d/d a_t, d/d a_p
};

__device__ inline Dual operator+(Dual x, Dual y) { return {x.v + y.v, x.a + y.a, x.b + y.b}; }
__device__ inline Dual operator-(Dual x, Dual y) { return {x.v - y.v, x.a - y.a, x.b - y.b}; }
__device__ inline Dual operator-(Dual x) { return {-x.v, -x.a, -x.b}; }
__device__ inline Dual operator*(Dual x, Dual y)
{
    return {x.v * y.v, x.a * y.v + x.v * y.a, x.b * y.v + x.v * y.b};
}
__device__ inline Dual operator*(double c, Dual x) { return {c * x.v, c * x.a, c * x.b}; }
__device__ inline Dual operator+(double c, Dual x) { return {c + x.v, x.a, x.b}; }
__device__ inline Dual operator-(double c, Dual x) { return {c - x.v, -x.a, -x.b}; }
__device__ inline Dual operator/(Dual x, Dual y)
{
    const double q = x.v / y.v;
    return {q, (x.a - q * y.a) / y.v, (x.b - q * y.b) / y.v};
}
__device__ inline Dual dsqrt(Dual x)
{
    const double r = sqrt(x.v);
    const double k = r > 0.0 ? 0.5 / r : 0.0;
    return {r, k * x.a, k * x.b};
}
__device__ inline Dual dsin(Dual x)
{
    double s, c;
    sincos(x.v, &s, &c);
    return {s, c * x.a, c * x.b};
}
__device__ inline Dual dcos(Dual x)
{
    double s, c;
    sincos(x.v, &s, &c);
    return {c, -s * x.a, -s * x.b};
}
__device__ inline Dual datan2(Dual y, Dual x)
{
    const double d = x.v * x.v + y.v * y.v;
    const double inv = d > 0.0 ? 1.0 / d : 0.0;
    return {atan2(y.v, x.v), (x.v * y.a - y.v * x.a) * inv, (x.v * y.b - y.v * x.b) * inv};
}

struct Deflected {
    Dual theta, dphi, chi;  // theta', phi' - phi, chi
};

// cos(a) and sin(a) / a as functions of q = a^2 (smooth at a = 0).
__device__ inline void cos_sinc(Dual q, Dual &cs, Dual &sc)
{
    if (q.v < 1e-4) {  // Taylor series; the first omitted terms are below 1e-26
        cs = 1.0 + q * (-0.5 + q * ((1.0 / 24) + q * ((-1.0 / 720) + (1.0 / 40320) * q)));
        sc = 1.0 + q * ((-1.0 / 6) + q * ((1.0 / 120) + q * ((-1.0 / 5040) + (1.0 / 362880) * q)));
    } else {
        const Dual a = dsqrt(q);
        cs = dcos(a);
        sc = dsin(a) / a;
    }
}

__device__ inline Deflected deflect_point(double theta, double at_v, double ap_v)
{
    double st, ct;
    sincos(theta, &st, &ct);
    const Dual at{at_v, 1.0, 0.0}, ap{ap_v, 0.0, 1.0};
    Dual cs, sc;
    cos_sinc(at * at + ap * ap, cs, sc);
    // n' in the rotated frame
    const Dual x = st * cs + ct * (sc * at);
    const Dual y = sc * ap;
    const Dual z = ct * cs - st * (sc * at);
    const Dual rho = dsqrt(x * x + y * y);
    Deflected d;
    d.theta = datan2(rho, z);
    d.dphi = datan2(y, x);
    // E1 = e_theta + k x e_theta + k x (k x e_theta) / (1 + cos a),
    // k = n x n' = sinc (a_t e_phi - a_p e_theta):
    //   k x e_theta = -sinc a_t n,  k x (k x e_theta) = -sinc^2 a_t (a_t e_theta + a_p e_phi)
    const Dual f = (sc * sc) / (1.0 + cs);
    const Dual sat = sc * at, fat = f * at;
    const Dual e1x = ct - st * sat - ct * (fat * at);
    const Dual e1y = -(fat * ap);
    const Dual e1z = -st - ct * sat + st * (fat * at);
    if (rho.v > 0.0) {
        // e_theta' = (z x, z y, -rho) / rho (x, y scaled), e_phi' = (-y, x, 0) / rho
        const Dual ut = (z * (x * e1x + y * e1y)) / rho - rho * e1z;
        const Dual up = (x * e1y - y * e1x) / rho;
        d.chi = -datan2(up, ut);
    } else {
        d.chi = Dual{0.0, 0.0, 0.0};
    }
    return d;
}

constexpr double kTwoPi = 6.283185307179586;

__device__ inline double wrap_phi(double p)
{
    if (p < 0.0)
        p += kTwoPi;
    if (p >= kTwoPi)
        p -= kTwoPi;
    return p;
}

template <typename T>
__global__ void deflect_kernel(const double *__restrict__ theta, const double *__restrict__ phi,
                               const T *__restrict__ alpha, int64_t npts,
                               double *__restrict__ theta_out, double *__restrict__ phi_out,
                               double *__restrict__ chi_out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += stride) {
        const Deflected d = deflect_point(theta[i], (double)alpha[i], (double)alpha[npts + i]);
        theta_out[i] = d.theta.v;
        phi_out[i] = wrap_phi(phi[i] + d.dphi.v);
        if (chi_out)
            chi_out[i] = d.chi.v;
    }
}

template <typename T>
__global__ void deflect_vjp_kernel(const double *__restrict__ theta, const T *__restrict__ alpha,
                                   int64_t npts, const double *__restrict__ g_theta,
                                   const double *__restrict__ g_phi,
                                   const double *__restrict__ g_chi, T *__restrict__ g_alpha)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += stride) {
        const Deflected d = deflect_point(theta[i], (double)alpha[i], (double)alpha[npts + i]);
        const double gt = g_theta ? g_theta[i] : 0.0;
        const double gp = g_phi ? g_phi[i] : 0.0;
        const double gc = g_chi ? g_chi[i] : 0.0;
        g_alpha[i] = (T)(gt * d.theta.a + gp * d.dphi.a + gc * d.chi.a);
        g_alpha[npts + i] = (T)(gt * d.theta.b + gp * d.dphi.b + gc * d.chi.b);
    }
}

// (Q + iU) <- e^{i sign s chi} (Q + iU)
template <typename T>
__global__ void spin_phase_kernel(T *__restrict__ map, const double *__restrict__ chi, int spin,
                                  int sign, int64_t npts)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += stride) {
        double s, c;
        sincos((double)(sign * spin) * chi[i], &s, &c);
        const double q = map[i], u = map[npts + i];
        map[i] = (T)(c * q - s * u);
        map[npts + i] = (T)(s * q + c * u);
    }
}

// For M = e^{i s chi} P and a real loss with gradient g = dL/dM (as (Q, U) pairs):
// dL/dP = e^{-i s chi} g and dL/dchi = s (g_U M_Q - g_Q M_U).
template <typename T>
__global__ void spin_phase_vjp_kernel(const T *__restrict__ g, const T *__restrict__ lensed,
                                      const double *__restrict__ chi, int spin, int64_t npts,
                                      T *__restrict__ g_unrot, double *__restrict__ g_chi)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += stride) {
        double s, c;
        sincos((double)spin * chi[i], &s, &c);
        const double gq = g[i], gu = g[npts + i];
        if (g_unrot) {
            g_unrot[i] = (T)(c * gq + s * gu);
            g_unrot[npts + i] = (T)(c * gu - s * gq);
        }
        if (g_chi)
            g_chi[i] = (double)spin * (gu * (double)lensed[i] - gq * (double)lensed[npts + i]);
    }
}

// out = f_l in for every stored coefficient of ncomp blocks, with
//   kind 0: f_l = sqrt(l (l + 1))                      (potential -> spin-1 deflection)
//   kind 1: f_l = l (l + 1) / 2                        (potential -> convergence)
//   kind 2: f_l = sqrt((l - 1) l (l + 1) (l + 2)) / 2  (potential -> spin-2 shear)
__device__ inline double l_factor(int kind, int l)
{
    const double L = (double)l;
    if (kind == 0)
        return sqrt(L * (L + 1.0));
    if (kind == 1)
        return 0.5 * L * (L + 1.0);
    return l >= 1 ? 0.5 * sqrt((L - 1.0) * L * (L + 1.0) * (L + 2.0)) : 0.0;
}

template <typename TC>
__global__ void alm_lscale_kernel(const TC *__restrict__ in, int lmax, int mmax, int ncomp,
                                  int64_t nalm, int kind, TC *__restrict__ out)
{
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax)
        return;
    const int64_t i = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
    const double f = l_factor(kind, l);
    for (int c = 0; c < ncomp; ++c) {
        TC v = in[c * nalm + i];
        v.x = (decltype(v.x))(f * (double)v.x);
        v.y = (decltype(v.y))(f * (double)v.y);
        out[c * nalm + i] = v;
    }
}

// Magnification determinant of the remapping n -> n' (Appendix B):
//   |A| = (sin a / a) ((1 - kappa)^2 + omega^2 - gamma^2)
//       + (cos a - sin a / a) (1 - kappa - cos(2 beta) gamma_1 - sin(2 beta) gamma_2),
// beta the direction of alpha from e_theta (cos 2 beta = (a_t^2 - a_p^2) / a^2, ...).
template <typename T>
__global__ void magnification_kernel(const T *__restrict__ alpha, const T *__restrict__ kappa,
                                     const T *__restrict__ omega, const T *__restrict__ gamma,
                                     int64_t npts, double *__restrict__ det)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += stride) {
        const double at = alpha[i], ap = alpha[npts + i];
        const double k = kappa[i], w = omega ? (double)omega[i] : 0.0;
        const double g1 = gamma[i], g2 = gamma[npts + i];
        const double q = at * at + ap * ap;
        double cs, sc;
        if (q < 1e-4) {
            cs = 1.0 + q * (-0.5 + q * ((1.0 / 24) + q * ((-1.0 / 720) + (1.0 / 40320) * q)));
            sc = 1.0 + q * ((-1.0 / 6) + q * ((1.0 / 120) + q * ((-1.0 / 5040) + (1.0 / 362880) * q)));
        } else {
            const double a = sqrt(q);
            double sa;
            sincos(a, &sa, &cs);
            sc = sa / a;
        }
        const double c2b = q > 0.0 ? (at * at - ap * ap) / q : 1.0;
        const double s2b = q > 0.0 ? 2.0 * at * ap / q : 0.0;
        det[i] = sc * ((1.0 - k) * (1.0 - k) + w * w - (g1 * g1 + g2 * g2)) +
                 (cs - sc) * (1.0 - k - c2b * g1 - s2b * g2);
    }
}

// out[c][i] = w[i] in[c][i] (quadrature weights applied to a map).
template <typename T>
__global__ void map_weight_kernel(const T *__restrict__ in, const double *__restrict__ w,
                                  int ncomp, int64_t npts, T *__restrict__ out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += stride) {
        const double wi = w[i];
        for (int c = 0; c < ncomp; ++c)
            out[c * npts + i] = (T)(wi * (double)in[c * npts + i]);
    }
}

unsigned elem_blocks(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

}  // namespace

hipError_t launch_deflect(const double *theta, const double *phi, const void *alpha, int prec,
                          int64_t npts, double *theta_out, double *phi_out, double *chi_out,
                          hipStream_t s)
{
    if (npts == 0)
        return hipSuccess;
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(deflect_kernel<double>, dim3(elem_blocks(npts)), dim3(256), 0, s, theta,
                           phi, (const double *)alpha, npts, theta_out, phi_out, chi_out);
    else
        hipLaunchKernelGGL(deflect_kernel<float>, dim3(elem_blocks(npts)), dim3(256), 0, s, theta,
                           phi, (const float *)alpha, npts, theta_out, phi_out, chi_out);
    return hipGetLastError();
}

hipError_t launch_deflect_vjp(const double *theta, const void *alpha, int prec, int64_t npts,
                              const double *g_theta, const double *g_phi, const double *g_chi,
                              void *g_alpha, hipStream_t s)
{
    if (npts == 0)
        return hipSuccess;
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(deflect_vjp_kernel<double>, dim3(elem_blocks(npts)), dim3(256), 0, s,
                           theta, (const double *)alpha, npts, g_theta, g_phi, g_chi,
                           (double *)g_alpha);
    else
        hipLaunchKernelGGL(deflect_vjp_kernel<float>, dim3(elem_blocks(npts)), dim3(256), 0, s,
                           theta, (const float *)alpha, npts, g_theta, g_phi, g_chi,
                           (float *)g_alpha);
    return hipGetLastError();
}

hipError_t launch_spin_phase(void *map, const double *chi, int spin, int sign, int prec,
                             int64_t npts, hipStream_t s)
{
    if (npts == 0)
        return hipSuccess;
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(spin_phase_kernel<double>, dim3(elem_blocks(npts)), dim3(256), 0, s,
                           (double *)map, chi, spin, sign, npts);
    else
        hipLaunchKernelGGL(spin_phase_kernel<float>, dim3(elem_blocks(npts)), dim3(256), 0, s,
                           (float *)map, chi, spin, sign, npts);
    return hipGetLastError();
}

hipError_t launch_spin_phase_vjp(const void *g, const void *lensed, const double *chi, int spin,
                                 int prec, int64_t npts, void *g_unrot, double *g_chi,
                                 hipStream_t s)
{
    if (npts == 0)
        return hipSuccess;
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(spin_phase_vjp_kernel<double>, dim3(elem_blocks(npts)), dim3(256), 0,
                           s, (const double *)g, (const double *)lensed, chi, spin, npts,
                           (double *)g_unrot, g_chi);
    else
        hipLaunchKernelGGL(spin_phase_vjp_kernel<float>, dim3(elem_blocks(npts)), dim3(256), 0, s,
                           (const float *)g, (const float *)lensed, chi, spin, npts,
                           (float *)g_unrot, g_chi);
    return hipGetLastError();
}

hipError_t launch_map_weight(const void *in, const double *w, int ncomp, int64_t npts, int prec,
                             void *out, hipStream_t s)
{
    if (npts == 0)
        return hipSuccess;
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(map_weight_kernel<double>, dim3(elem_blocks(npts)), dim3(256), 0, s,
                           (const double *)in, w, ncomp, npts, (double *)out);
    else
        hipLaunchKernelGGL(map_weight_kernel<float>, dim3(elem_blocks(npts)), dim3(256), 0, s,
                           (const float *)in, w, ncomp, npts, (float *)out);
    return hipGetLastError();
}

hipError_t launch_alm_lscale(const void *in, int lmax, int mmax, int ncomp, int kind, int prec,
                             void *out, hipStream_t s)
{
    const int64_t nalm = (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
    dim3 blk(256), grd((lmax + 1 + 255) / 256, mmax + 1);
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(alm_lscale_kernel<double2>, grd, blk, 0, s, (const double2 *)in, lmax,
                           mmax, ncomp, nalm, kind, (double2 *)out);
    else
        hipLaunchKernelGGL(alm_lscale_kernel<float2>, grd, blk, 0, s, (const float2 *)in, lmax,
                           mmax, ncomp, nalm, kind, (float2 *)out);
    return hipGetLastError();
}

hipError_t launch_magnification(const void *alpha, const void *kappa, const void *omega,
                                const void *gamma, int prec, int64_t npts, double *det,
                                hipStream_t s)
{
    if (npts == 0)
        return hipSuccess;
    if (prec == GSHT_F64)
        hipLaunchKernelGGL(magnification_kernel<double>, dim3(elem_blocks(npts)), dim3(256), 0, s,
                           (const double *)alpha, (const double *)kappa, (const double *)omega,
                           (const double *)gamma, npts, det);
    else
        hipLaunchKernelGGL(magnification_kernel<float>, dim3(elem_blocks(npts)), dim3(256), 0, s,
                           (const float *)alpha, (const float *)kappa, (const float *)omega,
                           (const float *)gamma, npts, det);
    return hipGetLastError();
}

}  // namespace gsht

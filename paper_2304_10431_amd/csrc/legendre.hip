// Legendre step of the general SHT on gfx950: "synthesis" (+ "doubling") and
// "adjoint synthesis" (+ "undoubling") of Sect. 3, in FP64.
//
// For each m and each ring pair (theta_j, pi - theta_j) of the equidistant grid
// theta_j = pi j / (ntheta - 1), one lane runs the three-term recurrence in l of
// the spin-weighted harmonic, normalised as p_l = sY_lm / N_l so that
//     p_{l+1} = (a_l cos(theta) + sigma b_l) p_l - p_{l-1},
// for both channels sigma = +s and sigma = -s.  The south ring reuses the north
// recurrence through sY_lm(pi - theta) = (-1)^(l+m) (-s)Y_lm(theta), and the
// column -m of a spin-s field through sY_{l,-m} = (-1)^(s+m) (-s)Y_lm.
//
// The start value at l0 = max(m, s) is a single half-angle power term that can
// be far below the double range; each channel carries a binary exponent offset
// (a non-positive multiple of 512) until its value has grown into range, and
// contributes nothing before that (such terms are below 2^-256 relative).
#include "gsht_internal.hpp"

#include <cmath>

namespace gsht {

template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };

// ---- host: start data ------------------------------------------------------

// sqrt((2 l0 + 1)/(4 pi) * X) as (mantissa, exponent) for X = v 2^e, in long double.
static void start_factor(long double v, long e, int l0, double *mant, int *ex)
{
    v *= (long double)(2 * l0 + 1) / (4.0L * 3.14159265358979323846264338327950288L);
    {
        int ee;
        v = frexpl(v, &ee);
        e += ee;
    }
    if (e & 1) {
        v *= 2.0L;
        e -= 1;
    }
    v = sqrtl(v);
    e /= 2;
    {
        int ee;
        v = frexpl(v, &ee);
        e += ee;
    }
    *mant = (double)v;
    *ex = (int)e;
}

std::vector<StartInfo> make_start_info(int lmax, int mmax, int spin)
{
    // Both channels' single Goldberg term at l0 = max(m, s) carries the binomial
    // X(m) = binom(2 l0, |m - s|) (binom(2 l0, m + s) for the channel -s is the same
    // number).  X(s) = 1, and one ratio per step gives the others:
    //   X(m + 1) = X(m) (2m + 2)(2m + 1) / ((m + 1 - s)(m + 1 + s))   (m >= s),
    //   X(m - 1) = X(m) (s + m) / (s - m + 1)                        (m <= s),
    // in long double with a separate binary exponent, O(mmax) in all.
    std::vector<long double> xv((size_t)mmax + 1);
    std::vector<long> xe((size_t)mmax + 1);
    auto renorm = [](long double &v, long &e) {
        int ee;
        v = frexpl(v, &ee);
        e += ee;
    };
    {
        long double v = 1.0L;
        long e = 0;
        if (spin <= mmax) {
            xv[(size_t)spin] = v;
            xe[(size_t)spin] = e;
        }
        for (int m = spin; m < mmax; ++m) {
            v *= (long double)(2 * m + 2) * (long double)(2 * m + 1) /
                 ((long double)(m + 1 - spin) * (long double)(m + 1 + spin));
            renorm(v, e);
            xv[(size_t)m + 1] = v;
            xe[(size_t)m + 1] = e;
        }
        v = 1.0L;
        e = 0;
        for (int m = spin; m > 0; --m) {
            v *= (long double)(spin + m) / (long double)(spin - m + 1);
            renorm(v, e);
            if (m - 1 <= mmax) {
                xv[(size_t)m - 1] = v;
                xe[(size_t)m - 1] = e;
            }
        }
    }
    std::vector<StartInfo> out((size_t)mmax + 1);
    for (int m = 0; m <= mmax; ++m) {
        StartInfo &si = out[(size_t)m];
        si.l0 = m > spin ? m : spin;
        si.pad = 0;
        double mant;
        int ex;
        start_factor(xv[(size_t)m], xe[(size_t)m], si.l0, &mant, &ex);
        for (int c = 0; c < 2; ++c) {
            const int sg = c == 0 ? spin : -spin;
            // single term of the Goldberg sum at l0: index r, half-angle exponents
            const int r = (m - sg) > 0 ? (m - sg) : 0;
            const int b = 2 * r + sg - m;
            const int a = 2 * si.l0 - b;
            const double mc = ((m + si.l0 - r - sg) & 1) != 0 ? -mant : mant;
            if (c == 0) {
                si.a_p = a; si.b_p = b; si.ex_p = ex; si.mant_p = mc;
            } else {
                si.a_m = a; si.b_m = b; si.ex_m = ex; si.mant_m = mc;
            }
        }
        (void)lmax;
    }
    return out;
}

// ---- device: recurrence tables ---------------------------------------------

// One thread per m: a_l, b_l and N_l for l0 <= l <= lmax (zeros below l0).
__global__ void leg_tables_kernel(int lmax, int mmax, int s, double2 *__restrict__ ab,
                                  double *__restrict__ norm)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m > mmax)
        return;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const int l0 = m > s ? m : s;
    for (int l = m; l < l0 && l <= lmax; ++l) {
        ab[base + l] = make_double2(0.0, 0.0);
        norm[base + l] = 0.0;
    }
    if (l0 > lmax)
        return;
    const double dm2 = (double)m * m, ds2 = (double)s * s;
    double nprev = 1.0, ncur = 1.0;  // N_{l-1}, N_l  (N_l0 = N_l0+1 = 1)
    norm[base + l0] = 1.0;
    for (int l = l0; l < lmax; ++l) {
        const double L = l;
        const double lp1sq = (L + 1) * (L + 1);
        const double inv = 1.0 / sqrt((lp1sq - dm2) * (lp1sq - ds2));
        const double ap = sqrt((2 * L + 3) / (2 * L + 1)) * (L + 1) * (2 * L + 1) * inv;
        double nnext;
        if (l == l0) {
            nnext = 1.0;
        } else {
            const double c3 = sqrt((2 * L + 3) / (2 * L - 1)) * (L + 1) * (2 * L + 1) * inv *
                              sqrt((L * L - dm2) * (L * L - ds2)) / (L * (2 * L + 1));
            nnext = c3 * nprev;
        }
        const double a = ap * ncur / nnext;
        const double b = (l == 0) ? 0.0 : a * (double)m * (double)s / (L * (L + 1));
        ab[base + l] = make_double2(a, b);
        norm[base + l + 1] = nnext;
        nprev = ncur;
        ncur = nnext;
    }
    ab[base + lmax] = make_double2(0.0, 0.0);
}

hipError_t launch_leg_tables(const gsht_plan &p, hipStream_t s)
{
    dim3 blk(64), grd((p.mmax + 1 + 63) / 64);
    hipLaunchKernelGGL(leg_tables_kernel, grd, blk, 0, s, p.lmax, p.mmax, p.spin, p.leg.ab,
                       p.leg.norm);
    return hipGetLastError();
}

// ---- device: coefficient preparation -----------------------------------------

// u = N_l * c_lm with the sign conventions folded in:
//   spin 0: u = a_lm (Im a_l0 dropped);  spin s: u+ = -(G + iC), u- = -(-1)^s (G* + i C*).
template <typename TC>
__global__ void prep_alm_kernel(const TC *__restrict__ alm, const double *__restrict__ norm,
                                int lmax, int mmax, int s, int64_t nalm, double mscale, int grad,
                                double *__restrict__ u)
{
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax)
        return;
    const int64_t i = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
    const double n = (l < s) ? 0.0 : (m > 0 ? mscale : 1.0) * norm[i];
    if (grad) {  // gradient-only spin s: u+ = -G (C = 0); u- follows in the kernel
        const TC gc = alm[i];
        u[2 * i] = -n * (double)gc.x;
        u[2 * i + 1] = (m == 0) ? 0.0 : -n * (double)gc.y;
    } else if (s == 0) {
        const TC a = alm[i];
        u[2 * i] = n * (double)a.x;
        u[2 * i + 1] = (m == 0) ? 0.0 : n * (double)a.y;
    } else {
        const TC gc = alm[i], cc = alm[nalm + i];
        const double gr = gc.x, gi = (m == 0) ? 0.0 : (double)gc.y;
        const double cr = cc.x, ci = (m == 0) ? 0.0 : (double)cc.y;
        const double sg = (s & 1) ? -1.0 : 1.0;
        u[4 * i + 0] = -n * (gr - ci);
        u[4 * i + 1] = -n * (gi + cr);
        u[4 * i + 2] = -sg * n * (gr + ci);
        u[4 * i + 3] = -sg * n * (cr - gi);
    }
}

hipError_t launch_prep_alm(const gsht_plan &p, const void *alm, double mscale, bool grad,
                           hipStream_t s)
{
    dim3 blk(256), grd((p.lmax + 1 + 255) / 256, p.mmax + 1);
    const int g = (grad && p.spin) ? 1 : 0;
    if (p.prec == GSHT_F64)
        hipLaunchKernelGGL(prep_alm_kernel<double2>, grd, blk, 0, s, (const double2 *)alm,
                           p.leg.norm, p.lmax, p.mmax, p.spin, p.nalm, mscale, g, p.uprep);
    else
        hipLaunchKernelGGL(prep_alm_kernel<float2>, grd, blk, 0, s, (const float2 *)alm,
                           p.leg.norm, p.lmax, p.mmax, p.spin, p.nalm, mscale, g, p.uprep);
    return hipGetLastError();
}

// Several maps: u[idx][k][US] for maps k < nm (interleaved per coefficient), each
// as prep_alm_kernel.  alm holds the nm maps one after the other ([nm][ncomp][nalm]).
template <typename TC>
__global__ void prep_multi_kernel(const TC *__restrict__ alm, const double *__restrict__ norm,
                                  int lmax, int mmax, int s, int64_t nalm, int nm,
                                  double *__restrict__ u)
{
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax)
        return;
    const int64_t i = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
    const double n = (l < s) ? 0.0 : norm[i];
    const int ncomp = s ? 2 : 1, us = s ? 4 : 2;
    for (int k = 0; k < nm; ++k) {
        const TC *a = alm + (int64_t)k * ncomp * nalm;
        double *o = u + ((int64_t)i * nm + k) * us;
        if (s == 0) {
            const TC c = a[i];
            o[0] = n * (double)c.x;
            o[1] = (m == 0) ? 0.0 : n * (double)c.y;
        } else {
            const TC gc = a[i], cc = a[nalm + i];
            const double gr = gc.x, gi = (m == 0) ? 0.0 : (double)gc.y;
            const double cr = cc.x, ci = (m == 0) ? 0.0 : (double)cc.y;
            const double sg = (s & 1) ? -1.0 : 1.0;
            o[0] = -n * (gr - ci);
            o[1] = -n * (gi + cr);
            o[2] = -sg * n * (gr + ci);
            o[3] = -sg * n * (cr - gi);
        }
    }
}

hipError_t launch_prep_multi(const gsht_plan &p, const void *alm, int nm, double *u, hipStream_t s)
{
    dim3 blk(256), grd((p.lmax + 1 + 255) / 256, p.mmax + 1);
    if (p.prec == GSHT_F64)
        hipLaunchKernelGGL(prep_multi_kernel<double2>, grd, blk, 0, s, (const double2 *)alm,
                           p.leg.norm, p.lmax, p.mmax, p.spin, p.nalm, nm, u);
    else
        hipLaunchKernelGGL(prep_multi_kernel<float2>, grd, blk, 0, s, (const float2 *)alm,
                           p.leg.norm, p.lmax, p.mmax, p.spin, p.nalm, nm, u);
    return hipGetLastError();
}

// Coefficient tiles of the matrix-core synthesis of NM = 8 NCB maps (FP32 plans),
// one workgroup per m.  First the largest |u| of each map's column m gives its
// scale 2^e (largest scaled value in [2^7, 2^8)) and oscale[m][map] = 2^-e;
// then every block kb of 16 degrees from l0 = max(m, s) gets, per type t (channel
// +s, -s), column block c, hi/lo part and lane, the 8 FP16 values of column
// n = lane % 32 (map 8 c + n / 4, entry n % 4) at degrees l0 + 16 kb + 8 (lane / 32) + j:
// channel +s: u0, u1, SG u2, SG u3; channel -s: u2, u3, SG u0, SG u1; spin 0: u0, u1,
// SG u0, SG u1 (u as prep_multi_kernel, SG = (-1)^(l - l0), zero past lmax and for maps
// >= nm).  The hi part is the FP16 rounding of the scaled value (through FP32), the lo
// part that of the remainder, both rounded towards zero.  Per block the 16 x 16
// (degree, map) coefficients are formed once (16 threads per map, consecutive
// degrees, so the reads coalesce) and staged in LDS for the tile writes.
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

__device__ inline void mfma_u(const float2 *__restrict__ alm, const double *__restrict__ norm,
                              int lmax, int m, int s, int64_t nalm, int map, int l, double *u)
{
    const int64_t i = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
    const double n = (l < s) ? 0.0 : norm[i];
    const int ncomp = s ? 2 : 1;
    const float2 *a = alm + (int64_t)map * ncomp * nalm;
    if (s == 0) {
        const float2 c = a[i];
        u[0] = n * (double)c.x;
        u[1] = (m == 0) ? 0.0 : n * (double)c.y;
        u[2] = u[3] = 0.0;
    } else {
        const float2 gc = a[i], cc = a[nalm + i];
        const double gr = gc.x, gi = (m == 0) ? 0.0 : (double)gc.y;
        const double cr = cc.x, ci = (m == 0) ? 0.0 : (double)cc.y;
        const double sg = (s & 1) ? -1.0 : 1.0;
        u[0] = -n * (gr - ci);
        u[1] = -n * (gi + cr);
        u[2] = -sg * n * (gr + ci);
        u[3] = -sg * n * (cr - gi);
    }
}

template <int NCB>
__global__ __launch_bounds__(256) void prep_mfma_kernel(const float2 *__restrict__ alm,
                                                        const double *__restrict__ norm, int lmax,
                                                        int s, int64_t nalm, int nm,
                                                        const int64_t *__restrict__ boff,
                                                        half8_t *__restrict__ Bt,
                                                        float *__restrict__ oscale)
{
    constexpr int NMX = 8 * NCB;
    const int m = blockIdx.x;
    const int l0 = m > s ? m : s;
    const int nt = s ? 2 : 1;
    const int tid = threadIdx.x;
    // thread -> (map, degree offset): 16 consecutive threads read 16 consecutive
    // degrees of one map
    const int tmap = tid / 16, tk = tid % 16;
    __shared__ unsigned mx[NMX];
    __shared__ double sc[NMX];
    __shared__ float U[NMX][4][16];  // scaled u of one block of 16 degrees
    if (tid < NMX)
        mx[tid] = 0u;
    __syncthreads();
    if (l0 <= lmax && tmap < nm) {
        float lm = 0.f;
        for (int l = l0 + tk; l <= lmax; l += 16) {
            double u[4];
            mfma_u(alm, norm, lmax, m, s, nalm, tmap, l, u);
            for (int c = 0; c < 4; ++c)
                lm = fmaxf(lm, (float)fabs(u[c]));
        }
        atomicMax(&mx[tmap], __float_as_uint(lm));  // non-negative floats order as integers
    }
    __syncthreads();
    if (tid < NMX) {
        const float v = __uint_as_float(mx[tid]);
        int e = 0;
        if (v > 0.f) {
            e = 7 - ilogbf(v);
            e = e < -100 ? -100 : (e > 100 ? 100 : e);
        }
        sc[tid] = ldexp(1.0, e);
        oscale[m * NMX + tid] = ldexpf(1.f, -e);
    }
    __syncthreads();
    if (l0 > lmax)
        return;
    const int nkb = (lmax - l0 + 16) / 16;
    const int per = nt * NCB * 2 * 64;
    half8_t *out = Bt + boff[m] * per;
    for (int kb = 0; kb < nkb; ++kb) {
        const int lb = l0 + 16 * kb;
        if (tmap < NMX) {
            double u[4] = {0.0, 0.0, 0.0, 0.0};
            if (tmap < nm && lb + tk <= lmax)
                mfma_u(alm, norm, lmax, m, s, nalm, tmap, lb + tk, u);
            for (int c = 0; c < 4; ++c)
                U[tmap][c][tk] = (float)(u[c] * sc[tmap]);
        }
        __syncthreads();
        for (int idx = tid; idx < per; idx += blockDim.x) {
            const int lane = idx % 64, hl = (idx / 64) % 2, c = (idx / 128) % NCB;
            const int t = idx / (128 * NCB);
            const int n = lane % 32, map = 8 * c + n / 4, e = n % 4;
            const int src = s == 0 ? (e & 1) : (t == 0 ? e : (e ^ 2));
            half8_t v;
            for (int j = 0; j < 8; ++j) {
                const int k = 8 * (lane / 32) + j;
                const float sg = (e >= 2 && ((lb + k - l0) & 1)) ? -1.f : 1.f;
                const float f = sg * U[map][src][k];
                const auto hp = __builtin_amdgcn_cvt_pkrtz(f, 0.f);
                v[j] = hl == 0 ? hp[0] : __builtin_amdgcn_cvt_pkrtz(f - (float)hp[0], 0.f)[0];
            }
            out[(int64_t)kb * per + idx] = v;
        }
        __syncthreads();
    }
}

hipError_t launch_prep_mfma(const gsht_plan &p, const void *alm, int nm, const int64_t *boff,
                            void *Bt, float *oscale, hipStream_t s)
{
    if (p.prec != GSHT_F32 || nm < 1 || nm > 16)
        return hipErrorInvalidValue;
    dim3 blk(256), grd(p.mmax + 1);
    if (nm > 8)
        hipLaunchKernelGGL(prep_mfma_kernel<2>, grd, blk, 0, s, (const float2 *)alm, p.leg.norm,
                           p.lmax, p.spin, p.nalm, nm, boff, (half8_t *)Bt, oscale);
    else
        hipLaunchKernelGGL(prep_mfma_kernel<1>, grd, blk, 0, s, (const float2 *)alm, p.leg.norm,
                           p.lmax, p.spin, p.nalm, nm, boff, (half8_t *)Bt, oscale);
    return hipGetLastError();
}

// S+-, N_l -> output coefficients (gradient/curl split for spin s).
template <typename TC>
__global__ void leg_finalize_kernel(const double *__restrict__ acc, const double *__restrict__ norm,
                                    int lmax, int mmax, int s, int64_t nalm, double mscale,
                                    int grad, TC *__restrict__ alm)
{
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax)
        return;
    const int64_t i = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
    const double n = (l < s) ? 0.0 : (m > 0 ? mscale : 1.0) * norm[i];
    TC o;
    if (grad) {  // gradient-only: acc holds S+ + (-1)^s S-, G = -(that) / 2
        o.x = -0.5 * n * acc[2 * i];
        o.y = (m == 0) ? 0.0 : -0.5 * n * acc[2 * i + 1];
        alm[i] = o;
    } else if (s == 0) {
        o.x = n * acc[2 * i];
        o.y = (m == 0) ? 0.0 : n * acc[2 * i + 1];
        alm[i] = o;
    } else {
        const double sg = (s & 1) ? -1.0 : 1.0;
        const double pr = n * acc[4 * i], pi = n * acc[4 * i + 1];
        const double mr = n * acc[4 * i + 2], mi = n * acc[4 * i + 3];
        TC gc, cc;
        gc.x = -0.5 * (pr + sg * mr);
        gc.y = (m == 0) ? 0.0 : -0.5 * (pi + sg * mi);
        cc.x = -0.5 * (pi - sg * mi);
        cc.y = (m == 0) ? 0.0 : 0.5 * (pr - sg * mr);
        alm[i] = gc;
        alm[nalm + i] = cc;
    }
}

hipError_t launch_leg_finalize(const gsht_plan &p, void *alm, double mscale, bool grad,
                               hipStream_t s)
{
    dim3 blk(256), grd((p.lmax + 1 + 255) / 256, p.mmax + 1);
    const int g = (grad && p.spin) ? 1 : 0;
    if (p.prec == GSHT_F64)
        hipLaunchKernelGGL(leg_finalize_kernel<double2>, grd, blk, 0, s, p.acc, p.leg.norm, p.lmax,
                           p.mmax, p.spin, p.nalm, mscale, g, (double2 *)alm);
    else
        hipLaunchKernelGGL(leg_finalize_kernel<float2>, grd, blk, 0, s, p.acc, p.leg.norm, p.lmax,
                           p.mmax, p.spin, p.nalm, mscale, g, (float2 *)alm);
    return hipGetLastError();
}

}  // namespace gsht

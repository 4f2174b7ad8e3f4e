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

// sqrt((2 l0 + 1)/(4 pi) * binom(2 l0, b)) as (mantissa, exponent), in long double.
static void start_factor(int l0, int b, double *mant, int *ex)
{
    int k = b < 2 * l0 - b ? b : 2 * l0 - b;
    long double v = 1.0L;
    long e = 0;
    for (int i = 1; i <= k; ++i) {
        int ee;
        v *= (long double)(2 * l0 - k + i) / (long double)i;
        v = frexpl(v, &ee);
        e += ee;
    }
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
    std::vector<StartInfo> out((size_t)mmax + 1);
    for (int m = 0; m <= mmax; ++m) {
        StartInfo &si = out[(size_t)m];
        si.l0 = m > spin ? m : spin;
        si.pad = 0;
        for (int c = 0; c < 2; ++c) {
            const int sg = c == 0 ? spin : -spin;
            // single term of the Goldberg sum at l0: index r, half-angle exponents
            const int r = (m - sg) > 0 ? (m - sg) : 0;
            const int b = 2 * r + sg - m;
            const int a = 2 * si.l0 - b;
            double mant;
            int ex;
            start_factor(si.l0, b, &mant, &ex);
            if (((m + si.l0 - r - sg) & 1) != 0)
                mant = -mant;
            if (c == 0) {
                si.a_p = a; si.b_p = b; si.ex_p = ex; si.mant_p = mant;
            } else {
                si.a_m = a; si.b_m = b; si.ex_m = ex; si.mant_m = mant;
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
                                int lmax, int mmax, int s, int64_t nalm, double *__restrict__ u)
{
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax)
        return;
    const int64_t i = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
    const double n = (l < s) ? 0.0 : norm[i];
    if (s == 0) {
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

hipError_t launch_prep_alm(const gsht_plan &p, const void *alm, hipStream_t s)
{
    dim3 blk(256), grd((p.lmax + 1 + 255) / 256, p.mmax + 1);
    if (p.prec == GSHT_F64)
        hipLaunchKernelGGL(prep_alm_kernel<double2>, grd, blk, 0, s, (const double2 *)alm,
                           p.leg.norm, p.lmax, p.mmax, p.spin, p.nalm, p.uprep);
    else
        hipLaunchKernelGGL(prep_alm_kernel<float2>, grd, blk, 0, s, (const float2 *)alm,
                           p.leg.norm, p.lmax, p.mmax, p.spin, p.nalm, p.uprep);
    return hipGetLastError();
}

// ---- device: start values and channel state -----------------------------------

struct XD {
    double m;
    int e;
};

__device__ inline void xnorm(XD &x)
{
    int k;
    x.m = frexp(x.m, &k);
    x.e += k;
}

// base^n (base >= 0, n >= 0) with a separate binary exponent; 0^0 = 1.
__device__ inline XD xpow(double base, int n)
{
    XD r{1.0, 0};
    if (n == 0)
        return r;
    if (base == 0.0)
        return XD{0.0, 0};
    XD b{base, 0};
    xnorm(b);
    while (n) {
        if (n & 1) {
            r.m *= b.m;
            r.e += b.e;
            xnorm(r);
        }
        b.m *= b.m;
        b.e *= 2;
        xnorm(b);
        n >>= 1;
    }
    return r;
}

constexpr double TWO_P256 = 1.157920892373162e77;  // 2^256

struct Chan {
    double p0, p1;  // p_{l-1}, p_l
    int ex;         // true value = p * 2^ex; ex == 0 <=> significant
};

__device__ inline Chan chan_init(double mant, int ex0, int a, int b, double sh, double ch)
{
    XD v{mant, ex0};
    XD ps = xpow(sh, a), pc = xpow(ch, b);
    v.m *= ps.m;
    v.e += ps.e;
    xnorm(v);
    v.m *= pc.m;
    v.e += pc.e;
    xnorm(v);
    Chan c;
    c.p0 = 0.0;
    if (v.m == 0.0) {
        c.p1 = 0.0;
        c.ex = 0;
    } else if (v.e >= -256) {
        c.p1 = ldexp(v.m, v.e);
        c.ex = 0;
    } else {
        const int t = v.e + 256;                      // < 0
        const int k = -((-t + 511) / 512);            // floor(t / 512)
        c.ex = 512 * k;
        c.p1 = ldexp(v.m, v.e - c.ex);
    }
    return c;
}

__device__ inline void chan_rescale(Chan &c)
{
    if (c.ex < 0 && fabs(c.p1) >= TWO_P256) {
        c.p0 = ldexp(c.p0, -512);
        c.p1 = ldexp(c.p1, -512);
        c.ex += 512;
    }
}

// ---- device: synthesis -----------------------------------------------------------

template <typename T> __device__ inline void store_c(typename cplx<T>::type *p, double re, double im)
{
    typename cplx<T>::type v;
    v.x = (T)re;
    v.y = (T)im;
    *p = v;
}

// Write ring value and, for interior rings, its doubled mirror with sign ms.
template <typename T>
__device__ inline void put_ring(typename cplx<T>::type *col, int j, int ntheta, int nd, double ms,
                                double re, double im)
{
    store_c<T>(col + j, re, im);
    if (j > 0 && j < ntheta - 1)
        store_c<T>(col + (nd - j), ms * re, ms * im);
}

// One wave per (m, chunk of 64 ring pairs); heavy m first.
template <typename T, bool SPIN>
__global__ __launch_bounds__(64) void leg_synth_kernel(
    const double2 *__restrict__ ab, const double *__restrict__ u, const StartInfo *__restrict__ st,
    int lmax, int mmax, int s, int ntheta, int nd, int npairs, int nchunk,
    typename cplx<T>::type *__restrict__ D)
{
    const int m = blockIdx.x / nchunk;
    const int chunk = blockIdx.x - m * nchunk;
    const int q = chunk * 64 + (int)threadIdx.x;
    const bool active = q < npairs;
    const StartInfo si = st[m];
    const int l0 = si.l0;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;

    const double t = active ? (double)q / (double)(ntheta - 1) : 0.5;
    const double x = cospi(t);
    const double sh = sinpi(0.5 * t), ch = cospi(0.5 * t);

    double npr = 0, npi = 0, spr = 0, spi = 0, nmr = 0, nmi = 0, smr = 0, smi = 0;
    if (l0 <= lmax) {
        Chan cp = chan_init(si.mant_p, si.ex_p, si.a_p, si.b_p, sh, ch);
        Chan cm = SPIN ? chan_init(si.mant_m, si.ex_m, si.a_m, si.b_m, sh, ch) : Chan{0, 0, 0};
        if (!active) {
            cp = Chan{0, 0, 0};
            cm = Chan{0, 0, 0};
        }
        int l = l0;
        // phase A: every channel of every lane below range -- recurrence only
        while (l <= lmax) {
            const bool sig = (cp.ex == 0) || (SPIN && cm.ex == 0);
            if (__any(sig))
                break;
            if (l < lmax) {
                const double2 c = ab[base + l];
                const double tp = fma(c.x, x, c.y);
                const double np = fma(tp, cp.p1, -cp.p0);
                cp.p0 = cp.p1;
                cp.p1 = np;
                if (SPIN) {
                    const double tm = fma(c.x, x, -c.y);
                    const double nm = fma(tm, cm.p1, -cm.p0);
                    cm.p0 = cm.p1;
                    cm.p1 = nm;
                }
                chan_rescale(cp);
                if (SPIN)
                    chan_rescale(cm);
            }
            ++l;
        }
        // phase B (masked) and C (all in range)
        while (l <= lmax) {
            const bool allsig = (cp.ex == 0) && (!SPIN || cm.ex == 0);
            const bool wave_all = __all(allsig);
            const double vp = (cp.ex == 0) ? cp.p1 : 0.0;
            const double vm = (SPIN && cm.ex == 0) ? cm.p1 : 0.0;
            const double sg = ((l - l0) & 1) ? -1.0 : 1.0;
            if (SPIN) {
                const double ur = u[4 * (base + l)], ui = u[4 * (base + l) + 1];
                const double wr = u[4 * (base + l) + 2], wi = u[4 * (base + l) + 3];
                npr = fma(ur, vp, npr);
                npi = fma(ui, vp, npi);
                spr = fma(sg * ur, vm, spr);
                spi = fma(sg * ui, vm, spi);
                nmr = fma(wr, vm, nmr);
                nmi = fma(wi, vm, nmi);
                smr = fma(sg * wr, vp, smr);
                smi = fma(sg * wi, vp, smi);
            } else {
                const double ur = u[2 * (base + l)], ui = u[2 * (base + l) + 1];
                npr = fma(ur, vp, npr);
                npi = fma(ui, vp, npi);
                spr = fma(sg * ur, vp, spr);
                spi = fma(sg * ui, vp, spi);
            }
            if (l < lmax) {
                const double2 c = ab[base + l];
                const double tp = fma(c.x, x, c.y);
                const double np = fma(tp, cp.p1, -cp.p0);
                cp.p0 = cp.p1;
                cp.p1 = np;
                if (SPIN) {
                    const double tm = fma(c.x, x, -c.y);
                    const double nm = fma(tm, cm.p1, -cm.p0);
                    cm.p0 = cm.p1;
                    cm.p1 = nm;
                }
                if (!wave_all) {
                    chan_rescale(cp);
                    if (SPIN)
                        chan_rescale(cm);
                }
            }
            ++l;
        }
    }
    if (!active)
        return;
    // south values carry (-1)^(l+m) = (-1)^(l0+m) (-1)^(l-l0)
    const double sfix = ((l0 + m) & 1) ? -1.0 : 1.0;
    const double ms = ((s + m) & 1) ? -1.0 : 1.0;
    const int jn = q, js = ntheta - 1 - q;
    typename cplx<T>::type *colp = D + (size_t)(SPIN ? m + mmax : m) * nd;
    put_ring<T>(colp, jn, ntheta, nd, ms, npr, npi);
    if (js != jn)
        put_ring<T>(colp, js, ntheta, nd, ms, sfix * spr, sfix * spi);
    if (SPIN && m > 0) {
        typename cplx<T>::type *colm = D + (size_t)(mmax - m) * nd;
        put_ring<T>(colm, jn, ntheta, nd, ms, nmr, nmi);
        if (js != jn)
            put_ring<T>(colm, js, ntheta, nd, ms, sfix * smr, sfix * smi);
    }
}

hipError_t launch_leg_synth(const gsht_plan &p, void *Dout, hipStream_t s)
{
    const int nchunk = (p.npairs + 63) / 64;
    dim3 blk(64), grd((unsigned)((p.mmax + 1) * nchunk));
    if (p.prec == GSHT_F64) {
        if (p.spin)
            hipLaunchKernelGGL((leg_synth_kernel<double, true>), grd, blk, 0, s, p.leg.ab, p.uprep,
                               p.leg.start, p.lmax, p.mmax, p.spin, p.ntheta, p.nd, p.npairs,
                               nchunk, (double2 *)Dout);
        else
            hipLaunchKernelGGL((leg_synth_kernel<double, false>), grd, blk, 0, s, p.leg.ab, p.uprep,
                               p.leg.start, p.lmax, p.mmax, p.spin, p.ntheta, p.nd, p.npairs,
                               nchunk, (double2 *)Dout);
    } else {
        if (p.spin)
            hipLaunchKernelGGL((leg_synth_kernel<float, true>), grd, blk, 0, s, p.leg.ab, p.uprep,
                               p.leg.start, p.lmax, p.mmax, p.spin, p.ntheta, p.nd, p.npairs,
                               nchunk, (float2 *)Dout);
        else
            hipLaunchKernelGGL((leg_synth_kernel<float, false>), grd, blk, 0, s, p.leg.ab, p.uprep,
                               p.leg.start, p.lmax, p.mmax, p.spin, p.ntheta, p.nd, p.npairs,
                               nchunk, (float2 *)Dout);
    }
    return hipGetLastError();
}

// ---- device: adjoint ------------------------------------------------------------

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        v += __shfl_xor(v, d, 64);
    return v;
}

template <typename T>
__device__ inline double2 ld_c(const typename cplx<T>::type *p)
{
    const typename cplx<T>::type v = *p;
    return make_double2((double)v.x, (double)v.y);
}

// Undoubled ring value H(j) from the doubled column.
template <typename T>
__device__ inline double2 ring_in(const typename cplx<T>::type *col, int j, int ntheta, int nd,
                                  double ms)
{
    double2 v = ld_c<T>(col + j);
    if (j > 0 && j < ntheta - 1) {
        const double2 w = ld_c<T>(col + (nd - j));
        v.x += ms * w.x;
        v.y += ms * w.y;
    }
    return v;
}

// One wave per (m, chunk of 64 ring pairs); per-l wave sums added atomically
// into acc[idx][0..3] = (S+ re, S+ im, S- re, S- im) (spin 0: [0..1]).
template <typename T, bool SPIN>
__global__ __launch_bounds__(64) void leg_adjoint_kernel(
    const double2 *__restrict__ ab, const StartInfo *__restrict__ st,
    const typename cplx<T>::type *__restrict__ D, int lmax, int mmax, int s, int ntheta, int nd,
    int npairs, int nchunk, double *__restrict__ acc)
{
    const int m = blockIdx.x / nchunk;
    const int chunk = blockIdx.x - m * nchunk;
    const int q = chunk * 64 + (int)threadIdx.x;
    const bool active = q < npairs;
    const StartInfo si = st[m];
    const int l0 = si.l0;
    if (l0 > lmax)
        return;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double t = active ? (double)q / (double)(ntheta - 1) : 0.5;
    const double x = cospi(t);
    const double sh = sinpi(0.5 * t), ch = cospi(0.5 * t);
    const double ms = ((s + m) & 1) ? -1.0 : 1.0;
    const double sfix = ((l0 + m) & 1) ? -1.0 : 1.0;
    const int jn = q, js = ntheta - 1 - q;

    double2 fpn = make_double2(0, 0), fps = fpn, fmn = fpn, fms = fpn;
    if (active) {
        const typename cplx<T>::type *colp = D + (size_t)(SPIN ? m + mmax : m) * nd;
        fpn = ring_in<T>(colp, jn, ntheta, nd, ms);
        if (js != jn) {
            fps = ring_in<T>(colp, js, ntheta, nd, ms);
            fps.x *= sfix;
            fps.y *= sfix;
        }
        if (SPIN) {
            const typename cplx<T>::type *colm = D + (size_t)(mmax - m) * nd;
            fmn = ring_in<T>(colm, jn, ntheta, nd, ms);
            if (js != jn) {
                fms = ring_in<T>(colm, js, ntheta, nd, ms);
                fms.x *= sfix;
                fms.y *= sfix;
            }
        }
    }
    Chan cp = chan_init(si.mant_p, si.ex_p, si.a_p, si.b_p, sh, ch);
    Chan cm = SPIN ? chan_init(si.mant_m, si.ex_m, si.a_m, si.b_m, sh, ch) : Chan{0, 0, 0};
    if (!active) {
        cp = Chan{0, 0, 0};
        cm = Chan{0, 0, 0};
    }
    for (int l = l0; l <= lmax; ++l) {
        const double vp = (cp.ex == 0) ? cp.p1 : 0.0;
        const double vm = (SPIN && cm.ex == 0) ? cm.p1 : 0.0;
        const bool any = __any(vp != 0.0 || vm != 0.0);
        if (any) {
            const double sg = ((l - l0) & 1) ? -1.0 : 1.0;
            double a0, a1, a2 = 0, a3 = 0;
            if (SPIN) {
                // S+ : Fp(N) p+ + sg Fp(S) p- ;  S- : conj(Fm(N)) p- + sg conj(Fm(S)) p+
                a0 = fpn.x * vp + sg * fps.x * vm;
                a1 = fpn.y * vp + sg * fps.y * vm;
                a2 = fmn.x * vm + sg * fms.x * vp;
                a3 = -(fmn.y * vm + sg * fms.y * vp);
            } else {
                a0 = (fpn.x + sg * fps.x) * vp;
                a1 = (fpn.y + sg * fps.y) * vp;
            }
            a0 = wave_sum(a0);
            a1 = wave_sum(a1);
            if (SPIN) {
                a2 = wave_sum(a2);
                a3 = wave_sum(a3);
            }
            if (threadIdx.x == 0) {
                double *dst = acc + (SPIN ? 4 : 2) * (base + l);
                unsafeAtomicAdd(dst, a0);
                unsafeAtomicAdd(dst + 1, a1);
                if (SPIN) {
                    unsafeAtomicAdd(dst + 2, a2);
                    unsafeAtomicAdd(dst + 3, a3);
                }
            }
        }
        if (l < lmax) {
            const double2 c = ab[base + l];
            const double tp = fma(c.x, x, c.y);
            const double np = fma(tp, cp.p1, -cp.p0);
            cp.p0 = cp.p1;
            cp.p1 = np;
            if (SPIN) {
                const double tm = fma(c.x, x, -c.y);
                const double nm = fma(tm, cm.p1, -cm.p0);
                cm.p0 = cm.p1;
                cm.p1 = nm;
            }
            chan_rescale(cp);
            if (SPIN)
                chan_rescale(cm);
        }
    }
}

hipError_t launch_leg_adjoint(const gsht_plan &p, const void *Din, hipStream_t s)
{
    const int nchunk = (p.npairs + 63) / 64;
    dim3 blk(64), grd((unsigned)((p.mmax + 1) * nchunk));
    hipError_t e = launch_zero(p.acc, sizeof(double) * (size_t)p.nalm * 2 * p.ncomp, s);
    if (e != hipSuccess)
        return e;
    if (p.prec == GSHT_F64) {
        if (p.spin)
            hipLaunchKernelGGL((leg_adjoint_kernel<double, true>), grd, blk, 0, s, p.leg.ab,
                               p.leg.start, (const double2 *)Din, p.lmax, p.mmax, p.spin, p.ntheta,
                               p.nd, p.npairs, nchunk, p.acc);
        else
            hipLaunchKernelGGL((leg_adjoint_kernel<double, false>), grd, blk, 0, s, p.leg.ab,
                               p.leg.start, (const double2 *)Din, p.lmax, p.mmax, p.spin, p.ntheta,
                               p.nd, p.npairs, nchunk, p.acc);
    } else {
        if (p.spin)
            hipLaunchKernelGGL((leg_adjoint_kernel<float, true>), grd, blk, 0, s, p.leg.ab,
                               p.leg.start, (const float2 *)Din, p.lmax, p.mmax, p.spin, p.ntheta,
                               p.nd, p.npairs, nchunk, p.acc);
        else
            hipLaunchKernelGGL((leg_adjoint_kernel<float, false>), grd, blk, 0, s, p.leg.ab,
                               p.leg.start, (const float2 *)Din, p.lmax, p.mmax, p.spin, p.ntheta,
                               p.nd, p.npairs, nchunk, p.acc);
    }
    return hipGetLastError();
}

// S+-, N_l -> output coefficients (gradient/curl split for spin s).
template <typename TC>
__global__ void leg_finalize_kernel(const double *__restrict__ acc, const double *__restrict__ norm,
                                    int lmax, int mmax, int s, int64_t nalm, TC *__restrict__ alm)
{
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax)
        return;
    const int64_t i = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
    const double n = (l < s) ? 0.0 : norm[i];
    TC o;
    if (s == 0) {
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

hipError_t launch_leg_finalize(const gsht_plan &p, void *alm, hipStream_t s)
{
    dim3 blk(256), grd((p.lmax + 1 + 255) / 256, p.mmax + 1);
    if (p.prec == GSHT_F64)
        hipLaunchKernelGGL(leg_finalize_kernel<double2>, grd, blk, 0, s, p.acc, p.leg.norm, p.lmax,
                           p.mmax, p.spin, p.nalm, (double2 *)alm);
    else
        hipLaunchKernelGGL(leg_finalize_kernel<float2>, grd, blk, 0, s, p.acc, p.leg.norm, p.lmax,
                           p.mmax, p.spin, p.nalm, (float2 *)alm);
    return hipGetLastError();
}

}  // namespace gsht

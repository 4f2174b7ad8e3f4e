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

// ---- device: start values ----------------------------------------------------------

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

// Start value of one channel at l0 as mant * 2^e (|mant| in [0.5, 1) or 0).
__device__ inline XD start_value(double mant, int ex0, int a, int b, double sh, double ch)
{
    XD v{mant, ex0};
    const XD ps = xpow(sh, a), pc = xpow(ch, b);
    v.m *= ps.m;
    v.e += ps.e;
    xnorm(v);
    v.m *= pc.m;
    v.e += pc.e;
    xnorm(v);
    return v;
}

constexpr double TWO_P256 = 0x1p256;
constexpr double TWO_M512 = 0x1p-512;

// Scaled representation used by the kernels: true value = p * 2^ex with ex a
// non-positive multiple of 512; ex == 0 means "in range" (|value| >= ~2^-256 when
// it got there), and only in-range values are accumulated.
__device__ inline void to_scaled(const XD &v, double &p, int &ex)
{
    if (v.m == 0.0) {
        p = 0.0;
        ex = 0;
    } else if (v.e >= -256) {
        p = ldexp(v.m, v.e);
        ex = 0;
    } else {
        const int t = v.e + 256;               // < 0
        ex = 512 * (-((-t + 511) / 512));      // 512 * floor(t / 512)
        p = ldexp(v.m, v.e - ex);
    }
}

// Ring pair geometry: theta_q = pi q / (ntheta - 1).
__device__ inline void ring_geom(int q, int ntheta, double &x, double &sh, double &ch)
{
    const double t = (double)q / (double)(ntheta - 1);
    x = cospi(t);
    sh = sinpi(0.5 * t);
    ch = cospi(0.5 * t);
}

// ---- device: live-chunk table ----------------------------------------------------

// For each (m, chunk), the first degree at which the chunk's most equatorial ring
// reaches 2^-900 in either channel (lmax + 1 if never).  Values of every other
// ring of the chunk are smaller there, so a chunk whose entry exceeds lmax has
// nothing above 2^-256 -- the accumulation threshold -- and is skipped.
template <bool SPIN>
__global__ void leg_live_kernel(const double2 *__restrict__ ab, const StartInfo *__restrict__ st,
                                int lmax, int mmax, int ntheta, int npairs, int chunk_pairs,
                                int nchunk, int32_t *__restrict__ lfirst)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)(mmax + 1) * nchunk)
        return;
    const int m = (int)(id / nchunk), c = (int)(id - (int64_t)(id / nchunk) * nchunk);
    const StartInfo si = st[m];
    const int l0 = si.l0;
    if (l0 > lmax) {
        lfirst[id] = lmax + 1;
        return;
    }
    int q = c * chunk_pairs + chunk_pairs - 1;
    if (q > npairs - 1)
        q = npairs - 1;
    double x, sh, ch;
    ring_geom(q, ntheta, x, sh, ch);
    const XD va = start_value(si.mant_p, si.ex_p, si.a_p, si.b_p, sh, ch);
    const XD vb = SPIN ? start_value(si.mant_m, si.ex_m, si.a_m, si.b_m, sh, ch) : XD{0.0, 0};
    // exact (mantissa, exponent) walk
    double a0 = 0, a1 = va.m, b0 = 0, b1 = vb.m;
    int ea = va.e, eb = vb.e;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    int res = lmax + 1;
    for (int l = l0; l <= lmax; ++l) {
        int k;
        const bool ha = a1 != 0.0 && (frexp(a1, &k), k + ea >= -900);
        const bool hb = SPIN && b1 != 0.0 && (frexp(b1, &k), k + eb >= -900);
        if (ha || hb) {
            res = l;
            break;
        }
        if (l == lmax)
            break;
        const double2 cf = ab[base + l];
        const double na = fma(fma(cf.x, x, cf.y), a1, -a0);
        a0 = a1;
        a1 = na;
        if (fabs(a1) > 0x1p64 || (a1 != 0.0 && fabs(a1) < 0x1p-64)) {
            frexp(a1, &k);
            a0 = ldexp(a0, -k);
            a1 = ldexp(a1, -k);
            ea += k;
        }
        if (SPIN) {
            const double nb = fma(fma(cf.x, x, -cf.y), b1, -b0);
            b0 = b1;
            b1 = nb;
            if (fabs(b1) > 0x1p64 || (b1 != 0.0 && fabs(b1) < 0x1p-64)) {
                frexp(b1, &k);
                b0 = ldexp(b0, -k);
                b1 = ldexp(b1, -k);
                eb += k;
            }
        }
    }
    lfirst[id] = res;
}

hipError_t launch_leg_live(const gsht_plan &p, hipStream_t s)
{
    const int64_t n = (int64_t)(p.mmax + 1) * p.leg_nchunk;
    dim3 blk(64), grd((unsigned)((n + 63) / 64));
    if (p.spin)
        hipLaunchKernelGGL(leg_live_kernel<true>, grd, blk, 0, s, p.leg.ab, p.leg.start, p.lmax,
                           p.mmax, p.ntheta, p.npairs, 64 * LEG_R, p.leg_nchunk, p.leg.lfirst);
    else
        hipLaunchKernelGGL(leg_live_kernel<false>, grd, blk, 0, s, p.leg.ab, p.leg.start, p.lmax,
                           p.mmax, p.ntheta, p.npairs, 64 * LEG_R, p.leg_nchunk, p.leg.lfirst);
    return hipGetLastError();
}

// ---- device: per-ring recurrence state ----------------------------------------------

// One ring pair: channel a = +s, channel b = -s (unused for spin 0).
struct Ring {
    double x;
    double a0, a1, b0, b1;  // p_{l-1}, p_l per channel
    int ea, eb;             // exponent offsets
};

__device__ inline Ring ring_init(const StartInfo &si, int q, int ntheta, bool active, bool spin)
{
    Ring r;
    double sh, ch;
    ring_geom(active ? q : 0, ntheta, r.x, sh, ch);
    r.a0 = r.b0 = 0.0;
    to_scaled(start_value(si.mant_p, si.ex_p, si.a_p, si.b_p, sh, ch), r.a1, r.ea);
    if (spin)
        to_scaled(start_value(si.mant_m, si.ex_m, si.a_m, si.b_m, sh, ch), r.b1, r.eb);
    else {
        r.b1 = 0.0;
        r.eb = 0;
    }
    if (!active) {
        r.a1 = r.b1 = 0.0;
        r.ea = r.eb = 0;
    }
    return r;
}

template <bool SPIN>
__device__ inline void ring_advance(Ring &r, double a, double b)
{
    const double ta = fma(a, r.x, b);
    const double na = fma(ta, r.a1, -r.a0);
    r.a0 = r.a1;
    r.a1 = na;
    if (SPIN) {
        const double tb = fma(a, r.x, -b);
        const double nb = fma(tb, r.b1, -r.b0);
        r.b0 = r.b1;
        r.b1 = nb;
    }
}

template <bool SPIN>
__device__ inline void ring_rescale(Ring &r)
{
    if (r.ea < 0 && fabs(r.a1) >= TWO_P256) {
        r.a0 *= TWO_M512;
        r.a1 *= TWO_M512;
        r.ea += 512;
    }
    if (SPIN && r.eb < 0 && fabs(r.b1) >= TWO_P256) {
        r.b0 *= TWO_M512;
        r.b1 *= TWO_M512;
        r.eb += 512;
    }
}

// Phase of a 64-ring slice (wave uniform): 0 = no ring in range, 1 = some,
// 2 = all in range (no masking, no rescaling needed any more).
template <bool SPIN>
__device__ inline int slice_phase(const Ring &r)
{
    const bool in = (r.ea == 0) && (!SPIN || r.eb == 0);
    const bool any = (r.ea == 0 && r.a1 != 0.0) || (SPIN && r.eb == 0 && r.b1 != 0.0);
    if (__all(in))
        return 2;
    return __any(any) ? 1 : 0;
}

// ---- device: synthesis ------------------------------------------------------------

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

// Accumulators of one ring pair: spin s -> N+ (0,1), S+ (2,3), N- (4,5), S- (6,7);
// spin 0 -> N (0,1), S (2,3).  SG = +1 / -1 is the parity sign (-1)^(l - l0).
template <bool SPIN, int SG>
__device__ inline void synth_acc(double (&c)[8], double va, double vb, double ur, double ui,
                                 double wr, double wi)
{
    c[0] = fma(ur, va, c[0]);
    c[1] = fma(ui, va, c[1]);
    if (SPIN) {
        c[2] = fma(SG * ur, vb, c[2]);
        c[3] = fma(SG * ui, vb, c[3]);
        c[4] = fma(wr, vb, c[4]);
        c[5] = fma(wi, vb, c[5]);
        c[6] = fma(SG * wr, va, c[6]);
        c[7] = fma(SG * wi, va, c[7]);
    } else {
        c[2] = fma(SG * ur, va, c[2]);
        c[3] = fma(SG * ui, va, c[3]);
    }
}

// One wave per (m, chunk of 64 R ring pairs); lane L of slice r handles ring pair
// q = chunk 64 R + 64 r + L.  Heavy m first.
template <typename T, bool SPIN, int R>
__global__ __launch_bounds__(64) void leg_synth_kernel(
    const double2 *__restrict__ ab, const double *__restrict__ u, const StartInfo *__restrict__ st,
    const int32_t *__restrict__ lfirst, int lmax, int mmax, int s, int ntheta, int nd, int npairs,
    int nchunk, typename cplx<T>::type *__restrict__ D)
{
    constexpr int US = SPIN ? 4 : 2;
    const int m = blockIdx.x / nchunk;
    const int chunk = blockIdx.x - m * nchunk;
    const int lane = threadIdx.x;
    const StartInfo si = st[m];
    const int l0 = si.l0;
    const bool live = (l0 <= lmax) && (lfirst[blockIdx.x] <= lmax);
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;

    Ring rg[R];
    double c[R][8];
    int ph[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = chunk * 64 * R + 64 * r + lane;
        rg[r] = ring_init(si, q, ntheta, live && q < npairs, SPIN);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            c[r][k] = 0.0;
        ph[r] = live ? slice_phase<SPIN>(rg[r]) : 2;
    }
    if (live) {
        int l = l0;
        for (; l + 1 <= lmax; l += 2) {
            const double2 c0 = ab[base + l];
            const double2 c1 = ab[base + l + 1];
            const double *u0 = u + US * (base + l);
            const double ur0 = u0[0], ui0 = u0[1], wr0 = SPIN ? u0[2] : 0, wi0 = SPIN ? u0[3] : 0;
            const double ur1 = u0[US], ui1 = u0[US + 1], wr1 = SPIN ? u0[US + 2] : 0,
                         wi1 = SPIN ? u0[US + 3] : 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Ring &g = rg[r];
                if (ph[r] == 2) {
                    synth_acc<SPIN, 1>(c[r], g.a1, g.b1, ur0, ui0, wr0, wi0);
                    ring_advance<SPIN>(g, c0.x, c0.y);
                    synth_acc<SPIN, -1>(c[r], g.a1, g.b1, ur1, ui1, wr1, wi1);
                    ring_advance<SPIN>(g, c1.x, c1.y);
                } else {
                    if (ph[r] == 1) {
                        const double va = g.ea == 0 ? g.a1 : 0.0, vb = g.eb == 0 ? g.b1 : 0.0;
                        synth_acc<SPIN, 1>(c[r], va, vb, ur0, ui0, wr0, wi0);
                    }
                    ring_advance<SPIN>(g, c0.x, c0.y);
                    if (ph[r] == 1) {
                        const double va = g.ea == 0 ? g.a1 : 0.0, vb = g.eb == 0 ? g.b1 : 0.0;
                        synth_acc<SPIN, -1>(c[r], va, vb, ur1, ui1, wr1, wi1);
                    }
                    ring_advance<SPIN>(g, c1.x, c1.y);
                    ring_rescale<SPIN>(g);
                    ph[r] = slice_phase<SPIN>(g);
                }
            }
        }
        if (l == lmax) {
            const double *u0 = u + US * (base + l);
            const double ur0 = u0[0], ui0 = u0[1], wr0 = SPIN ? u0[2] : 0, wi0 = SPIN ? u0[3] : 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const Ring &g = rg[r];
                const double va = g.ea == 0 ? g.a1 : 0.0, vb = g.eb == 0 ? g.b1 : 0.0;
                synth_acc<SPIN, 1>(c[r], va, vb, ur0, ui0, wr0, wi0);
            }
        }
    }
    // south values carry (-1)^(l+m) = (-1)^(l0+m) (-1)^(l-l0)
    const double sfix = ((l0 + m) & 1) ? -1.0 : 1.0;
    const double ms = ((s + m) & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = chunk * 64 * R + 64 * r + lane;
        if (q >= npairs)
            continue;
        const int jn = q, js = ntheta - 1 - q;
        typename cplx<T>::type *colp = D + (size_t)(SPIN ? m + mmax : m) * nd;
        put_ring<T>(colp, jn, ntheta, nd, ms, c[r][0], c[r][1]);
        if (js != jn)
            put_ring<T>(colp, js, ntheta, nd, ms, sfix * c[r][2], sfix * c[r][3]);
        if (SPIN && m > 0) {
            typename cplx<T>::type *colm = D + (size_t)(mmax - m) * nd;
            put_ring<T>(colm, jn, ntheta, nd, ms, c[r][4], c[r][5]);
            if (js != jn)
                put_ring<T>(colm, js, ntheta, nd, ms, sfix * c[r][6], sfix * c[r][7]);
        }
    }
}

hipError_t launch_leg_synth(const gsht_plan &p, void *Dout, hipStream_t s)
{
    dim3 blk(64), grd((unsigned)((p.mmax + 1) * p.leg_nchunk));
#define GSHT_LEG_SYNTH(T, SP, C)                                                                 \
    hipLaunchKernelGGL((leg_synth_kernel<T, SP, LEG_R>), grd, blk, 0, s, p.leg.ab, p.uprep,      \
                       p.leg.start, p.leg.lfirst, p.lmax, p.mmax, p.spin, p.ntheta, p.nd, p.npairs, \
                       p.leg_nchunk, (C *)Dout)
    if (p.prec == GSHT_F64) {
        if (p.spin) GSHT_LEG_SYNTH(double, true, double2);
        else GSHT_LEG_SYNTH(double, false, double2);
    } else {
        if (p.spin) GSHT_LEG_SYNTH(float, true, float2);
        else GSHT_LEG_SYNTH(float, false, float2);
    }
#undef GSHT_LEG_SYNTH
    return hipGetLastError();
}

// ---- device: adjoint -------------------------------------------------------------------

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

// Per-ring adjoint inputs.  Spin 0: e = F(N) + F(S'), o = F(N) - F(S') (even / odd
// l - l0).  Spin s: F+(N), F+(S'), conj F-(N), conj F-(S') with S' = (-1)^(l0+m) S.
struct RingIn {
    double v[8];
};

// Contribution of one ring to the per-degree sums cb[0..NC-1]:
//   spin s: S+ += a F+(N) + SG b F+(S'),  S- += b cF-(N) + SG a cF-(S')
//   spin 0: b_l += a (SG > 0 ? e : o)
template <bool SPIN, int SG>
__device__ inline void adj_acc(double *cb, const RingIn &in, double va, double vb)
{
    if (SPIN) {
        cb[0] = fma(va, in.v[0], cb[0]);
        cb[1] = fma(va, in.v[1], cb[1]);
        cb[0] = fma(SG * vb, in.v[2], cb[0]);
        cb[1] = fma(SG * vb, in.v[3], cb[1]);
        cb[2] = fma(vb, in.v[4], cb[2]);
        cb[3] = fma(vb, in.v[5], cb[3]);
        cb[2] = fma(SG * va, in.v[6], cb[2]);
        cb[3] = fma(SG * va, in.v[7], cb[3]);
    } else {
        cb[0] = fma(va, in.v[SG > 0 ? 0 : 2], cb[0]);
        cb[1] = fma(va, in.v[SG > 0 ? 1 : 3], cb[1]);
    }
}

// One wave per (m, chunk of 64 R ring pairs).  Every 8 degrees, the per-lane sums
// are transposed through LDS, reduced over the 64 lanes and added to
// acc[idx][0..NC-1] with one coalesced FP64 atomic per (degree, component).
template <typename T, bool SPIN, int R>
__global__ __launch_bounds__(64) void leg_adjoint_kernel(
    const double2 *__restrict__ ab, const StartInfo *__restrict__ st,
    const int32_t *__restrict__ lfirst, const typename cplx<T>::type *__restrict__ D, int lmax,
    int mmax, int s, int ntheta, int nd, int npairs, int nchunk, double *__restrict__ acc)
{
    constexpr int NC = SPIN ? 4 : 2;
    constexpr int B = 8;
    constexpr int V = B * NC;
    __shared__ double red[V * 64];
    const int m = blockIdx.x / nchunk;
    const int chunk = blockIdx.x - m * nchunk;
    const int lane = threadIdx.x;
    const StartInfo si = st[m];
    const int l0 = si.l0;
    if (l0 > lmax || lfirst[blockIdx.x] > lmax)
        return;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double ms = ((s + m) & 1) ? -1.0 : 1.0;
    const double sfix = ((l0 + m) & 1) ? -1.0 : 1.0;

    Ring rg[R];
    RingIn in[R];
    int ph[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = chunk * 64 * R + 64 * r + lane;
        const bool active = q < npairs;
        rg[r] = ring_init(si, q, ntheta, active, SPIN);
        ph[r] = slice_phase<SPIN>(rg[r]);
        double2 fpn = make_double2(0, 0), fps = fpn, fmn = fpn, fms = fpn;
        if (active) {
            const int jn = q, js = ntheta - 1 - q;
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
        if (SPIN) {
            in[r].v[0] = fpn.x; in[r].v[1] = fpn.y;
            in[r].v[2] = fps.x; in[r].v[3] = fps.y;
            in[r].v[4] = fmn.x; in[r].v[5] = -fmn.y;
            in[r].v[6] = fms.x; in[r].v[7] = -fms.y;
        } else {
            in[r].v[0] = fpn.x + fps.x; in[r].v[1] = fpn.y + fps.y;
            in[r].v[2] = fpn.x - fps.x; in[r].v[3] = fpn.y - fps.y;
            in[r].v[4] = in[r].v[5] = in[r].v[6] = in[r].v[7] = 0.0;
        }
    }

    for (int lb = l0; lb <= lmax; lb += B) {
        double cb[V];
#pragma unroll
        for (int k = 0; k < V; ++k)
            cb[k] = 0.0;
#pragma unroll
        for (int b = 0; b < B; b += 2) {
            const int l = lb + b;
            if (l > lmax)
                break;
            const double2 c0 = ab[base + l];
            const bool two = l + 1 <= lmax;
            const double2 c1 = two ? ab[base + l + 1] : make_double2(0.0, 0.0);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                Ring &g = rg[r];
                if (ph[r] == 2) {
                    adj_acc<SPIN, 1>(cb + b * NC, in[r], g.a1, g.b1);
                    ring_advance<SPIN>(g, c0.x, c0.y);
                    if (two) {
                        adj_acc<SPIN, -1>(cb + (b + 1) * NC, in[r], g.a1, g.b1);
                        ring_advance<SPIN>(g, c1.x, c1.y);
                    }
                } else {
                    if (ph[r] == 1) {
                        const double va = g.ea == 0 ? g.a1 : 0.0, vb = g.eb == 0 ? g.b1 : 0.0;
                        adj_acc<SPIN, 1>(cb + b * NC, in[r], va, vb);
                    }
                    ring_advance<SPIN>(g, c0.x, c0.y);
                    if (two) {
                        if (ph[r] == 1) {
                            const double va = g.ea == 0 ? g.a1 : 0.0, vb = g.eb == 0 ? g.b1 : 0.0;
                            adj_acc<SPIN, -1>(cb + (b + 1) * NC, in[r], va, vb);
                        }
                        ring_advance<SPIN>(g, c1.x, c1.y);
                    }
                    ring_rescale<SPIN>(g);
                    ph[r] = slice_phase<SPIN>(g);
                }
            }
        }
        bool active = false;
#pragma unroll
        for (int r = 0; r < R; ++r)
            active = active || ph[r] != 0;
        if (!active)
            continue;  // every slice still below range: the block's sums are zero
        // transpose through LDS (rotated columns), reduce over lanes, add atomically
        __syncthreads();
#pragma unroll
        for (int v = 0; v < V; ++v)
            red[v * 64 + ((lane + v) & 63)] = cb[v];
        __syncthreads();
        constexpr int H = 64 / V;
        constexpr int SPAN = 64 / H;
        const int v = lane % V, h = lane / V;
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < SPAN; ++i)
            sum += red[v * 64 + ((h * SPAN + i + v) & 63)];
#pragma unroll
        for (int d = V; d < 64; d <<= 1)
            sum += __shfl_xor(sum, d, 64);
        if (lane < V && lb + lane / NC <= lmax)
            unsafeAtomicAdd(acc + (base + lb) * NC + lane, sum);
    }
}

hipError_t launch_leg_adjoint(const gsht_plan &p, const void *Din, hipStream_t s)
{
    dim3 blk(64), grd((unsigned)((p.mmax + 1) * p.leg_nchunk));
    hipError_t e = launch_zero(p.acc, sizeof(double) * (size_t)p.nalm * 2 * p.ncomp, s);
    if (e != hipSuccess)
        return e;
#define GSHT_LEG_ADJ(T, SP, C)                                                                   \
    hipLaunchKernelGGL((leg_adjoint_kernel<T, SP, LEG_R>), grd, blk, 0, s, p.leg.ab, p.leg.start, \
                       p.leg.lfirst, (const C *)Din, p.lmax, p.mmax, p.spin, p.ntheta, p.nd,      \
                       p.npairs, p.leg_nchunk, p.acc)
    if (p.prec == GSHT_F64) {
        if (p.spin) GSHT_LEG_ADJ(double, true, double2);
        else GSHT_LEG_ADJ(double, false, double2);
    } else {
        if (p.spin) GSHT_LEG_ADJ(float, true, float2);
        else GSHT_LEG_ADJ(float, false, float2);
    }
#undef GSHT_LEG_ADJ
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

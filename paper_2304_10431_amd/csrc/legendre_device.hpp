// Device helpers shared by the Legendre kernels (single-map, several-map and
// matrix-core forms): start values with a separate binary exponent, the per-ring
// recurrence state and its range handling, the XCD-aware work mapping and the
// doubled-column stores.  The conventions are described in legendre_kernels.hip.
#pragma once

#include <type_traits>

#include "gsht_internal.hpp"

namespace gsht {

template <typename T> struct cplxk;
template <> struct cplxk<float> { using type = float2; };
template <> struct cplxk<double> { using type = double2; };

// ---- start values -----------------------------------------------------------------

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

// One channel's value at l0: mant 2^ex0 sin(theta/2)^a cos(theta/2)^b.
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
// In-range thresholds 2^INX: values from there up are held unscaled (normal
// doubles; in the decaying region the recurrence only grows them).  The synthesis
// takes 2^-900, which ends its masked phase early; the adjoint takes 2^-256, which
// spares it the lane reductions of blocks that hold only negligible terms.
constexpr int SYN_IN_EXP = -900;
constexpr int ADJ_IN_EXP = -256;

// true value = p 2^ex, ex a non-positive multiple of 512, ex == 0 <=> in range.
template <int INX>
__device__ inline void to_scaled(const XD &v, double &p, int &ex)
{
    if (v.m == 0.0) {
        p = 0.0;
        ex = 0;
    } else if (v.e >= INX + 1) {
        p = ldexp(v.m, v.e);
        ex = 0;
    } else {
        const int t = v.e + 256;              // < 0
        ex = 512 * (-((-t + 511) / 512));     // 512 floor(t / 512)
        p = ldexp(v.m, v.e - ex);
    }
}

__device__ inline void ring_geom(int q, int ntheta, double &x, double &sh, double &ch)
{
    const double t = (double)q / (double)(ntheta - 1);
    x = cospi(t);
    sh = sinpi(0.5 * t);
    ch = cospi(0.5 * t);
}

// ---- work mapping -------------------------------------------------------------------

// Workgroups are dispatched round-robin over the MI355X's 8 XCDs.  All chunks of one
// m are kept on one XCD, so that XCD's L2 serves the m's coefficient stream to all of
// them (spread over every XCD, each 4 MB L2 would hold dozens of streams and thrash),
// and the m values are dealt to the XCDs round-robin, largest work first on each.
constexpr int NXCD = 8;

__device__ inline void xcd_map(int nchunk, int &m, int &chunk)
{
    const int x = blockIdx.x % NXCD, k = blockIdx.x / NXCD;
    const int g = k / nchunk;
    chunk = k - g * nchunk;
    m = x + NXCD * g;
}

inline unsigned xcd_grid(int mmax, int nchunk)
{
    return (unsigned)(NXCD * ((mmax + NXCD) / NXCD) * nchunk);
}

// ---- per-ring recurrence state ------------------------------------------------------

struct Ring {
    double x;
    double a0, a1, b0, b1;  // p_{l-1}, p_l of channels +s and -s
    int ea, eb;             // exponent offsets
};

template <int INX>
__device__ inline Ring ring_init(const StartInfo &si, int q, int ntheta, bool active, bool spin)
{
    Ring r;
    double sh, ch;
    ring_geom(active ? q : 0, ntheta, r.x, sh, ch);
    r.a0 = r.b0 = 0.0;
    to_scaled<INX>(start_value(si.mant_p, si.ex_p, si.a_p, si.b_p, sh, ch), r.a1, r.ea);
    if (spin)
        to_scaled<INX>(start_value(si.mant_m, si.ex_m, si.a_m, si.b_m, sh, ch), r.b1, r.eb);
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

// A scaled channel whose true value p 2^e has reached 2^INX is folded to e = 0;
// otherwise it is rescaled by 2^-512 once |p| reaches 2^256.  Selects only, no
// lane-divergent branch (the matrix-core kernels schedule their products among the
// recurrence steps; the vector kernels run the same code, at equal speed and bits).
// A fold happens only at e = -512 or -1024 (values reach at most 2^288 before the
// next check), where 2^e is still a double, so the product by it is exact like ldexp.
template <int INX>
__device__ inline void rescale_channel(double &p0, double &p1, int &e)
{
    const bool neg = e < 0;
    const bool fold = neg && fabs(p1) >= ldexp(1.0, INX - e);
    const bool down = neg && !fold && fabs(p1) >= TWO_P256;
    const double f = fold ? ldexp(1.0, e) : (down ? TWO_M512 : 1.0);
    p0 *= f;
    p1 *= f;
    e = fold ? 0 : (down ? e + 512 : e);
}

template <bool SPIN, int INX>
__device__ inline void ring_rescale(Ring &r)
{
    rescale_channel<INX>(r.a0, r.a1, r.ea);
    if (SPIN)
        rescale_channel<INX>(r.b0, r.b1, r.eb);
}

// Wave-uniform slice state: 0 = no lane in range, 1 = some, 2 = all.
template <bool SPIN>
__device__ inline int slice_phase(const Ring &r)
{
    const bool in = (r.ea == 0) && (!SPIN || r.eb == 0);
    const bool some = (r.ea == 0 && r.a1 != 0.0) || (SPIN && r.eb == 0 && r.b1 != 0.0);
    if (__all(in))
        return 2;
    return __any(some) ? 1 : 0;
}

// Silent blocks: while no lane of the wave holds a channel in range every term would
// get the weight 0, so only the recurrence runs (no sums, no reductions), with the
// rescaling and the slice phases after every 8 degrees (the longest interval between
// checks the growth bound of the rescaling allows).  ab_m points at the
// degree-indexed coefficients of the wave's m; lb advances.
template <bool SPIN, int INX, int R>
__device__ inline void silent_blocks(Ring (&rg)[R], const double2 *ab_m, int &lb, int lmax,
                                     bool &all_in, bool &some_in)
{
    for (; lb + 7 <= lmax && !some_in; lb += 8) {
        const double2 *abl = ab_m + lb;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const double2 cc = abl[b];
#pragma unroll
            for (int r = 0; r < R; ++r)
                ring_advance<SPIN>(rg[r], cc.x, cc.y);
        }
        all_in = true;
        some_in = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ring_rescale<SPIN, INX>(rg[r]);
            const int p = slice_phase<SPIN>(rg[r]);
            all_in = all_in && p == 2;
            some_in = some_in || p != 0;
        }
    }
}

template <bool B>
using flag = std::integral_constant<bool, B>;

// ---- synthesis -------------------------------------------------------------------

template <typename T>
__device__ inline void store_c(typename cplxk<T>::type *p, double re, double im)
{
    typename cplxk<T>::type v;
    v.x = (T)re;
    v.y = (T)im;
    *p = v;
}

// Ring value and, for interior rings, its doubled mirror with sign ms.
template <typename T>
__device__ inline void put_ring(typename cplxk<T>::type *col, int j, int ntheta, int nd, double ms,
                                double re, double im)
{
    store_c<T>(col + j, re, im);
    if (j > 0 && j < ntheta - 1)
        store_c<T>(col + (nd - j), ms * re, ms * im);
}

template <typename T>
__device__ inline double2 ld_c(const typename cplxk<T>::type *p)
{
    const typename cplxk<T>::type v = *p;
    return make_double2((double)v.x, (double)v.y);
}

// Undoubled ring value H(j) from the doubled column.
template <typename T>
__device__ inline double2 ring_in(const typename cplxk<T>::type *col, int j, int ntheta, int nd,
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

}  // namespace gsht

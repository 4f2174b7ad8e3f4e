// Legendre recurrence kernels of the general SHT on gfx950: the "synthesis" and
// "doubling" steps of Sect. 3 and their adjoints ("undoubling" and "adjoint
// synthesis"), FP64 throughout.
//
// For each m and each ring pair (theta_q, pi - theta_q) of the equidistant grid
// theta_q = pi q / (ntheta - 1), one lane runs the three-term recurrence in l of
// the spin-weighted harmonic, normalised as p_l = sY_lm / N_l so that
//     p_{l+1} = (a_l cos(theta) + sigma b_l) p_l - p_{l-1},
// for both channels sigma = +s (a) and sigma = -s (b).  The south ring reuses the
// north recurrence through sY_lm(pi - theta) = (-1)^(l+m) (-s)Y_lm(theta), and the
// column -m of a spin-s field through sY_{l,-m} = (-1)^(s+m) (-s)Y_lm.
//
// Start values at l0 = max(m, s) can lie far below the double range: each channel
// carries an exponent offset e (a non-positive multiple of 512), the true value
// being p 2^e, and contributes only while e = 0.  A channel reaches e = 0 once its
// true value passes 2^-900 (synthesis) or 2^-256 (adjoint), checked at block ends,
// so terms smaller than that, relative to the O(1) values of the oscillating
// region, are dropped.
//
// Work decomposition: one wave per (m, chunk); a chunk is R slices of 64
// consecutive ring pairs, lane L of slice r owning pair 64 (R chunk + r) + L.
// Degrees advance in blocks of 8; offsets change only at block ends.  A block runs
// "masked" (out-of-range channels excluded for the whole block, rescaling and
// phase update at its end) until every lane of the wave is in range; from then on
// blocks run without masks or checks, and only a final partial block checks the
// degree bound.  Chunks whose most equatorial ring stays below 2^-900 up to lmax
// are skipped outright.
#include "legendre_device.hpp"

namespace gsht {

// ---- live-chunk table -------------------------------------------------------------

// For each (m, chunk): the first degree at which the chunk's most equatorial ring
// reaches 2^THR in either channel (lmax + 1 if never).  The other rings of the
// chunk are smaller there, so a chunk whose entry exceeds lmax has nothing at or
// above 2^THR and is skipped.  THR is the kernel's in-range threshold: the synthesis
// takes 2^-900 and the adjoint 2^-256, below which it adds nothing (a channel
// contributes only once its value has reached that threshold), so skipping such a
// chunk leaves the results unchanged.
template <bool SPIN>
__global__ void leg_live_kernel(const double2 *__restrict__ ab, const StartInfo *__restrict__ st,
                                int lmax, int mmax, int ntheta, int npairs, int chunk_pairs,
                                int nchunk, int thr, int32_t *__restrict__ lfirst)
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
    double a0 = 0, a1 = va.m, b0 = 0, b1 = vb.m;
    int ea = va.e, eb = vb.e;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    int res = lmax + 1;
    for (int l = l0; l <= lmax; ++l) {
        int k;
        const bool ha = a1 != 0.0 && (frexp(a1, &k), k + ea >= thr);
        const bool hb = SPIN && b1 != 0.0 && (frexp(b1, &k), k + eb >= thr);
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

static void live_launch(const gsht_plan &p, int r, int nchunk, int thr, int32_t *lfirst,
                        hipStream_t s)
{
    const int64_t n = (int64_t)(p.mmax + 1) * nchunk;
    dim3 blk(64), grd((unsigned)((n + 63) / 64));
    if (p.spin)
        hipLaunchKernelGGL(leg_live_kernel<true>, grd, blk, 0, s, p.leg.ab, p.leg.start, p.lmax,
                           p.mmax, p.ntheta, p.npairs, 64 * r, nchunk, thr, lfirst);
    else
        hipLaunchKernelGGL(leg_live_kernel<false>, grd, blk, 0, s, p.leg.ab, p.leg.start, p.lmax,
                           p.mmax, p.ntheta, p.npairs, 64 * r, nchunk, thr, lfirst);
}

hipError_t launch_leg_live(const gsht_plan &p, hipStream_t s)
{
    live_launch(p, p.syn_r, p.syn_nchunk, SYN_IN_EXP, p.leg.lfirst_syn, s);
    live_launch(p, p.adj_r, p.adj_nchunk, ADJ_IN_EXP, p.leg.lfirst_adj, s);
    return hipGetLastError();
}

hipError_t launch_leg_live_adj(const gsht_plan &p, hipStream_t s)
{
    live_launch(p, p.adj_r, p.adj_nchunk, ADJ_IN_EXP, p.leg.lfirst_adj, s);
    return hipGetLastError();
}

// Accumulators of one ring pair: spin s -> N+ (0,1), S+ (2,3), N- (4,5), S- (6,7);
// spin 0 -> N (0,1), S (2,3).  SG = (-1)^(l - l0).
template <bool SPIN, int SG>
__device__ inline void synth_acc(double (&c)[8], double va, double vb, const double *u)
{
    c[0] = fma(u[0], va, c[0]);
    c[1] = fma(u[1], va, c[1]);
    if (SPIN) {
        c[2] = fma(SG * u[0], vb, c[2]);
        c[3] = fma(SG * u[1], vb, c[3]);
        c[4] = fma(u[2], vb, c[4]);
        c[5] = fma(u[3], vb, c[5]);
        c[6] = fma(SG * u[2], va, c[6]);
        c[7] = fma(SG * u[3], va, c[7]);
    } else {
        c[2] = fma(SG * u[0], va, c[2]);
        c[3] = fma(SG * u[1], va, c[3]);
    }
}

// Gradient-only spin s (C = 0): u- = (-1)^s conj(u+), so the four ring sums follow
// from the products of u+ with both channels, kept per degree parity:
// E_a (0,1), E_b (2,3) for SG = +1 and O_a (4,5), O_b (6,7) for SG = -1;
//   N+ = E_a + O_a,  S+ = E_b - O_b,  N- = (-1)^s conj(E_b + O_b),
//   S- = (-1)^s conj(E_a - O_a)
// (4 FMA per ring pair and degree instead of 8).
template <int SG>
__device__ inline void synth_acc_grad(double (&c)[8], double va, double vb, const double *u)
{
    constexpr int o = SG > 0 ? 0 : 4;
    c[o + 0] = fma(u[0], va, c[o + 0]);
    c[o + 1] = fma(u[1], va, c[o + 1]);
    c[o + 2] = fma(u[0], vb, c[o + 2]);
    c[o + 3] = fma(u[1], vb, c[o + 3]);
}

template <bool SPIN, bool GRAD, int SG>
__device__ inline void synth_acc_any(double (&c)[8], double va, double vb, const double *u)
{
    if constexpr (GRAD)
        synth_acc_grad<SG>(c, va, vb, u);
    else
        synth_acc<SPIN, SG>(c, va, vb, u);
}

// Add a masked block's sums t to c for the channels in range (the offsets are
// those the block ran with: rescaling happens after the fold).  Channel +s feeds
// c[0,1,6,7], channel -s c[2..5]; spin 0 has channel +s only.  Gradient-only:
// channel +s feeds c[0,1,4,5], channel -s c[2,3,6,7].
template <bool SPIN, bool GRAD = false>
__device__ inline void synth_fold(double (&c)[8], const double (&t)[8], const Ring &r)
{
    const bool ia = r.ea == 0, ib = SPIN && r.eb == 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const bool chan_a = GRAD ? ((k & 2) == 0) : (!SPIN || k < 2 || k > 5);
        const bool in = chan_a ? ia : ib;
        c[k] += in ? t[k] : 0.0;
    }
}

constexpr int LB = 8;  // degrees per block

// Waves per SIMD each synthesis shape is compiled for: R = 2 fits 96 registers, five
// waves (about 1 % faster than four at 124 registers; a few values spill around the
// loops, none inside them).
template <int R>
constexpr int syn_waves()
{
    return R == 2 ? 5 : 1;
}

template <typename T, bool SPIN, int R, bool GRAD = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(syn_waves<R>())))
void leg_synth_kernel(
    const double2 *__restrict__ ab, const double *__restrict__ u, const StartInfo *__restrict__ st,
    const int32_t *__restrict__ lfirst, int lmax, int mmax, int s, int ntheta, int nd, int npairs,
    int nchunk, typename cplxk<T>::type *__restrict__ D)
{
    static_assert(SPIN || !GRAD, "gradient-only needs spin > 0");
    constexpr int US = (SPIN && !GRAD) ? 4 : 2;
    int m, chunk;
    xcd_map(nchunk, m, chunk);
    if (m > mmax)
        return;
    const int lane = threadIdx.x;
    const StartInfo si = st[m];
    const int l0 = si.l0;
    const bool live = (l0 <= lmax) && (lfirst[m * nchunk + chunk] <= lmax);
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;

    Ring rg[R];
    double c[R][8];
    bool all_in = true, some_in = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = chunk * 64 * R + 64 * r + lane;
        rg[r] = ring_init<SYN_IN_EXP>(si, q, ntheta, live && q < npairs, SPIN);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            c[r][k] = 0.0;
        const int ph = slice_phase<SPIN>(rg[r]);
        all_in = all_in && ph == 2;
        some_in = some_in || ph != 0;
    }
    // Masked block: the block's terms are summed separately and added only for
    // channels in range (offset 0, constant inside a block); then rescaling and the
    // slice phases.  Only the final partial block (TAIL) checks the degree bound.
    auto masked_block = [&](int lb, auto tail) {
        constexpr bool TAIL = decltype(tail)::value;
        const double2 *abl = ab + base + lb;
        const double *ul = u + US * (base + lb);
        double t[R][8];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < 8; ++k)
                t[r][k] = 0.0;
        // two rolled halves: a fully unrolled block would load all its scalar
        // coefficients at once and run out of scalar registers
#pragma unroll 1
        for (int h = 0; h < LB; h += LB / 2)
#pragma unroll
        for (int b = h; b < h + LB / 2; b += 2) {
            const int l = lb + b;
            if (TAIL && l > lmax)
                break;
            const double2 c0 = abl[b];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                synth_acc_any<SPIN, GRAD, 1>(t[r], rg[r].a1, rg[r].b1, ul + US * b);
                ring_advance<SPIN>(rg[r], c0.x, c0.y);
            }
            if (TAIL && l + 1 > lmax)
                break;
            const double2 c1 = abl[b + 1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                synth_acc_any<SPIN, GRAD, -1>(t[r], rg[r].a1, rg[r].b1, ul + US * (b + 1));
                ring_advance<SPIN>(rg[r], c1.x, c1.y);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            synth_fold<SPIN, GRAD>(c[r], t[r], rg[r]);
        all_in = true;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ring_rescale<SPIN, SYN_IN_EXP>(rg[r]);
            all_in = all_in && (slice_phase<SPIN>(rg[r]) == 2);
        }
    };
    if (live) {
        // Sequential loops (no loop-carried value crosses a branch merge): silent
        // blocks until some lane is in range, masked full blocks until every lane is,
        // full plain blocks, and a masked partial tail.
        int lb = l0;
        silent_blocks<SPIN, SYN_IN_EXP>(rg, ab + base, lb, lmax, all_in, some_in);
        for (; lb + LB - 1 <= lmax && !all_in; lb += LB)
            masked_block(lb, flag<false>());
        // Full plain blocks, run as degree pairs whose coefficients are loaded one
        // pair ahead, so that the scalar loads overlap the previous pair's arithmetic.
        if (lb + LB - 1 <= lmax) {
            const int lend = lb + ((lmax - lb + 1) / LB) * LB;
            struct Pair {
                double2 c0, c1;
                double u[2 * US];
            };
            auto load_pair = [&](int l) {
                Pair q;
                q.c0 = ab[base + l];
                q.c1 = ab[base + l + 1];
#pragma unroll
                for (int k = 0; k < 2 * US; ++k)
                    q.u[k] = u[US * (base + l) + k];
                return q;
            };
            Pair cur = load_pair(lb);
#pragma unroll 4
            for (; lb < lend; lb += 2) {
                const Pair nxt = load_pair(lb + 2 < lend ? lb + 2 : lb);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    synth_acc_any<SPIN, GRAD, 1>(c[r], rg[r].a1, rg[r].b1, cur.u);
                    ring_advance<SPIN>(rg[r], cur.c0.x, cur.c0.y);
                    synth_acc_any<SPIN, GRAD, -1>(c[r], rg[r].a1, rg[r].b1, cur.u + US);
                    ring_advance<SPIN>(rg[r], cur.c1.x, cur.c1.y);
                }
                cur = nxt;
            }
        }
        if (lb <= lmax)
            masked_block(lb, flag<true>());
    }
    // south values carry (-1)^(l+m) = (-1)^(l0+m) (-1)^(l-l0)
    const double sfix = ((l0 + m) & 1) ? -1.0 : 1.0;
    const double ms = ((s + m) & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = chunk * 64 * R + 64 * r + lane;
        if (q >= npairs)
            continue;
        if constexpr (GRAD) {  // parity sums -> N+, S+, N-, S- (see synth_acc_grad)
            const double sg = (s & 1) ? -1.0 : 1.0;
            double (&v)[8] = c[r];
            const double ea0 = v[0], ea1 = v[1], eb0 = v[2], eb1 = v[3];
            const double oa0 = v[4], oa1 = v[5], ob0 = v[6], ob1 = v[7];
            v[0] = ea0 + oa0;
            v[1] = ea1 + oa1;
            v[2] = eb0 - ob0;
            v[3] = eb1 - ob1;
            v[4] = sg * (eb0 + ob0);
            v[5] = -sg * (eb1 + ob1);
            v[6] = sg * (ea0 - oa0);
            v[7] = -sg * (ea1 - oa1);
        }
        const int jn = q, js = ntheta - 1 - q;
        typename cplxk<T>::type *colp = D + (size_t)(SPIN ? m + mmax : m) * nd;
        put_ring<T>(colp, jn, ntheta, nd, ms, c[r][0], c[r][1]);
        if (js != jn)
            put_ring<T>(colp, js, ntheta, nd, ms, sfix * c[r][2], sfix * c[r][3]);
        if (SPIN && m > 0) {
            typename cplxk<T>::type *colm = D + (size_t)(mmax - m) * nd;
            put_ring<T>(colm, jn, ntheta, nd, ms, c[r][4], c[r][5]);
            if (js != jn)
                put_ring<T>(colm, js, ntheta, nd, ms, sfix * c[r][6], sfix * c[r][7]);
        }
    }
}

template <int R>
static void synth_launch(const gsht_plan &p, void *Dout, bool grad, hipStream_t s)
{
    dim3 blk(64), grd(xcd_grid(p.mmax, p.syn_nchunk));
#define GSHT_LEG_SYNTH(T, SP, G, C)                                                              \
    hipLaunchKernelGGL((leg_synth_kernel<T, SP, R, G>), grd, blk, 0, s, p.leg.ab, p.uprep,       \
                       p.leg.start, p.leg.lfirst_syn, p.lmax, p.mmax, p.spin, p.ntheta, p.nd,     \
                       p.npairs, p.syn_nchunk, (C *)Dout)
    if (p.prec == GSHT_F64) {
        if (p.spin && grad) GSHT_LEG_SYNTH(double, true, true, double2);
        else if (p.spin) GSHT_LEG_SYNTH(double, true, false, double2);
        else GSHT_LEG_SYNTH(double, false, false, double2);
    } else {
        if (p.spin && grad) GSHT_LEG_SYNTH(float, true, true, float2);
        else if (p.spin) GSHT_LEG_SYNTH(float, true, false, float2);
        else GSHT_LEG_SYNTH(float, false, false, float2);
    }
#undef GSHT_LEG_SYNTH
}

hipError_t launch_leg_synth(const gsht_plan &p, void *Dout, bool grad, hipStream_t s)
{
    switch (p.syn_r) {
    case 1: synth_launch<1>(p, Dout, grad, s); break;
    case 2: synth_launch<2>(p, Dout, grad, s); break;
    case 4: synth_launch<4>(p, Dout, grad, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- synthesis of several maps sharing one geometry --------------------------------

// NM maps at once: the recurrence (both channels) runs once per ring pair and
// degree and feeds the sums of every map; coefficients are interleaved per degree
// as u[idx][map][US].  Masked blocks weight the Legendre values by 0/1 per channel
// (offset 0 or not, constant inside a block) instead of keeping block sums.  The
// chunking (R slices of 64 ring pairs) is the single-map kernel's, so the dead-chunk
// table is shared.  Map k's doubled columns start at D + k dstride.
template <typename T, bool SPIN, int R, int NM>
__global__ __launch_bounds__(64) void leg_synth_multi_kernel(
    const double2 *__restrict__ ab, const double *__restrict__ u, const StartInfo *__restrict__ st,
    const int32_t *__restrict__ lfirst, int lmax, int mmax, int s, int ntheta, int nd, int npairs,
    int nchunk, size_t dstride, typename cplxk<T>::type *__restrict__ D)
{
    constexpr int US = SPIN ? 4 : 2;
    constexpr int UD = NM * US;  // doubles per degree
    int m, chunk;
    xcd_map(nchunk, m, chunk);
    if (m > mmax)
        return;
    const int lane = threadIdx.x;
    const StartInfo si = st[m];
    const int l0 = si.l0;
    const bool live = (l0 <= lmax) && (lfirst[m * nchunk + chunk] <= lmax);
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;

    Ring rg[R];
    double c[R][NM][8];
    bool all_in = true;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = chunk * 64 * R + 64 * r + lane;
        rg[r] = ring_init<SYN_IN_EXP>(si, q, ntheta, live && q < npairs, SPIN);
#pragma unroll
        for (int k = 0; k < NM; ++k)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                c[r][k][j] = 0.0;
        all_in = all_in && (slice_phase<SPIN>(rg[r]) == 2);
    }
    auto masked_block = [&](int lb, auto tail) {
        constexpr bool TAIL = decltype(tail)::value;
        double wa[R], wb[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            wa[r] = rg[r].ea == 0 ? 1.0 : 0.0;
            wb[r] = (SPIN && rg[r].eb == 0) ? 1.0 : 0.0;
        }
#pragma unroll 1
        for (int b = 0; b < LB; b += 2) {
            const int l = lb + b;
            if (TAIL && l > lmax)
                break;
            const double2 c0 = ab[base + l];
            const double *u0 = u + UD * (base + l);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double va = rg[r].a1 * wa[r], vb = rg[r].b1 * wb[r];
#pragma unroll
                for (int k = 0; k < NM; ++k)
                    synth_acc<SPIN, 1>(c[r][k], va, vb, u0 + US * k);
                ring_advance<SPIN>(rg[r], c0.x, c0.y);
            }
            if (TAIL && l + 1 > lmax)
                break;
            const double2 c1 = ab[base + l + 1];
            const double *u1 = u0 + UD;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double va = rg[r].a1 * wa[r], vb = rg[r].b1 * wb[r];
#pragma unroll
                for (int k = 0; k < NM; ++k)
                    synth_acc<SPIN, -1>(c[r][k], va, vb, u1 + US * k);
                ring_advance<SPIN>(rg[r], c1.x, c1.y);
            }
        }
        all_in = true;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ring_rescale<SPIN, SYN_IN_EXP>(rg[r]);
            all_in = all_in && (slice_phase<SPIN>(rg[r]) == 2);
        }
    };
    if (live) {
        int lb = l0;
        for (; lb + LB - 1 <= lmax && !all_in; lb += LB)
            masked_block(lb, flag<false>());
        const int lend = lb + ((lmax - lb + 1) / LB) * LB;
#pragma unroll 1
        for (; lb < lend; lb += 2) {
            const double2 c0 = ab[base + lb], c1 = ab[base + lb + 1];
            const double *u0 = u + UD * (base + lb);
#pragma unroll
            for (int r = 0; r < R; ++r) {
#pragma unroll
                for (int k = 0; k < NM; ++k)
                    synth_acc<SPIN, 1>(c[r][k], rg[r].a1, rg[r].b1, u0 + US * k);
                ring_advance<SPIN>(rg[r], c0.x, c0.y);
#pragma unroll
                for (int k = 0; k < NM; ++k)
                    synth_acc<SPIN, -1>(c[r][k], rg[r].a1, rg[r].b1, u0 + UD + US * k);
                ring_advance<SPIN>(rg[r], c1.x, c1.y);
            }
        }
        if (lb <= lmax)
            masked_block(lb, flag<true>());
    }
    const double sfix = ((l0 + m) & 1) ? -1.0 : 1.0;
    const double ms = ((s + m) & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = chunk * 64 * R + 64 * r + lane;
        if (q >= npairs)
            continue;
        const int jn = q, js = ntheta - 1 - q;
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            typename cplxk<T>::type *Dk = D + k * dstride;
            typename cplxk<T>::type *colp = Dk + (size_t)(SPIN ? m + mmax : m) * nd;
            put_ring<T>(colp, jn, ntheta, nd, ms, c[r][k][0], c[r][k][1]);
            if (js != jn)
                put_ring<T>(colp, js, ntheta, nd, ms, sfix * c[r][k][2], sfix * c[r][k][3]);
            if (SPIN && m > 0) {
                typename cplxk<T>::type *colm = Dk + (size_t)(mmax - m) * nd;
                put_ring<T>(colm, jn, ntheta, nd, ms, c[r][k][4], c[r][k][5]);
                if (js != jn)
                    put_ring<T>(colm, js, ntheta, nd, ms, sfix * c[r][k][6], sfix * c[r][k][7]);
            }
        }
    }
}

template <int R, int NM>
static void synth_multi_launch(const gsht_plan &p, const double *u, void *Dout, size_t dstride,
                               hipStream_t s)
{
    dim3 blk(64), grd(xcd_grid(p.mmax, p.syn_nchunk));
#define GSHT_LEG_SYNTH_M(T, SP, C)                                                               \
    hipLaunchKernelGGL((leg_synth_multi_kernel<T, SP, R, NM>), grd, blk, 0, s, p.leg.ab, u,      \
                       p.leg.start, p.leg.lfirst_syn, p.lmax, p.mmax, p.spin, p.ntheta, p.nd,     \
                       p.npairs, p.syn_nchunk, dstride, (C *)Dout)
    if (p.prec == GSHT_F64) {
        if (p.spin) GSHT_LEG_SYNTH_M(double, true, double2);
        else GSHT_LEG_SYNTH_M(double, false, double2);
    } else {
        if (p.spin) GSHT_LEG_SYNTH_M(float, true, float2);
        else GSHT_LEG_SYNTH_M(float, false, float2);
    }
#undef GSHT_LEG_SYNTH_M
}

// nm maps (2 or 4) at once; slices per lane as the plan's synthesis (1 or 2).
hipError_t launch_leg_synth_multi(const gsht_plan &p, int nm, const double *u, void *Dout,
                                  size_t dstride, hipStream_t s)
{
    const int key = 10 * p.syn_r + nm;
    switch (key) {
    case 12: synth_multi_launch<1, 2>(p, u, Dout, dstride, s); break;
    case 14: synth_multi_launch<1, 4>(p, u, Dout, dstride, s); break;
    case 22: synth_multi_launch<2, 2>(p, u, Dout, dstride, s); break;
    case 24: synth_multi_launch<2, 4>(p, u, Dout, dstride, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- adjoint -----------------------------------------------------------------------

// Per-ring adjoint inputs.  Spin 0: e = F(N) + F(S'), o = F(N) - F(S') (even / odd
// l - l0).  Spin s: F+(N), F+(S'), conj F-(N), conj F-(S'), S' = (-1)^(l0+m) S.
struct RingIn {
    double v[8];
};

// One ring's contribution to the per-degree sums cb[0..NC-1]:
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

// Gradient-only spin s: only T = S+ + (-1)^s S- is needed (G = -T / 2).  With the
// ring inputs precombined as X = F+(N) + SG sg cF-(S'), Y = SG F+(S') + sg cF-(N)
// (sg = (-1)^s, one pair per degree parity SG), T += a X + b Y; a and b go to
// separate sums (0,1) and (2,3), added before the lane reduction.
template <int SG>
__device__ inline void adj_acc_grad(double *cb, const RingIn &in, double va, double vb)
{
    constexpr int o = SG > 0 ? 0 : 2;
    cb[0] = fma(va, in.v[o + 0], cb[0]);
    cb[1] = fma(va, in.v[o + 1], cb[1]);
    cb[2] = fma(vb, in.v[o + 4], cb[2]);
    cb[3] = fma(vb, in.v[o + 5], cb[3]);
}

template <bool SPIN, bool GRAD, int SG>
__device__ inline void adj_acc_any(double *cb, const RingIn &in, double va, double vb)
{
    if constexpr (GRAD)
        adj_acc_grad<SG>(cb, in, va, vb);
    else
        adj_acc<SPIN, SG>(cb, in, va, vb);
}

// a' = [a(0..31), b(0..31)], b' = [a(32..63), b(32..63)] (v_permlane32_swap on both
// halves of the doubles); returns a' + b': lanes 0..31 hold a summed over lanes L
// and L + 32, lanes 32..63 hold b summed likewise.
__device__ inline double swap_add32(double a, double b)
{
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32),
                                                     false, false);
    const double a2 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    const double b2 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
    return a2 + b2;
}

// Same with v_permlane16_swap (odd rows of a <-> even rows of b): rows 0 and 2 end
// with a summed over rows (0,1) resp. (2,3), rows 1 and 3 with b likewise.
__device__ inline double swap_add16(double a, double b)
{
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32),
                                                     false, false);
    const double a2 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    const double b2 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
    return a2 + b2;
}

// Degrees per masked block of the adjoint (blocks before every lane is in range): the
// masked blocks set the kernel's register count, and at 4 degrees the R = 3 shapes fit
// 168 registers, three waves per SIMD (9.43 ms at the benchmark against 9.55 for
// 8-degree masked blocks at two waves, and 10.18 for 4-degree ones at two waves).
constexpr int ADJ_MASKED_B = 4;

// Waves per SIMD each adjoint shape is compiled for.
template <int R, int B>
constexpr int adj_waves()
{
    return R == 3 ? 3 : 1;
}

// One wave per (m, chunk).  Per block of B degrees the V = B NC per-lane sums are
// reduced over the 64 lanes: two swap-add stages in registers leave V/4 values per
// lane, each value spread over the 16 lanes of one row; these go through LDS
// (rotated slots, conflict free) and are summed by V groups of 64/V lanes.  The
// results are added to acc[idx][0..NC-1] with one coalesced FP64 atomic per
// (degree, component).
template <typename T, bool SPIN, int R, int B, bool GRAD = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(adj_waves<R, B>())))
void leg_adjoint_kernel(
    const double2 *__restrict__ ab, const StartInfo *__restrict__ st,
    const int32_t *__restrict__ lfirst, const typename cplxk<T>::type *__restrict__ D, int lmax,
    int mmax, int s, int ntheta, int nd, int npairs, int nchunk, double *__restrict__ acc)
{
    static_assert(SPIN || !GRAD, "gradient-only needs spin > 0");
    constexpr int NC = SPIN ? 4 : 2;         // per-lane sums per degree
    constexpr int NR = GRAD ? 2 : NC;        // reduced values per degree
    constexpr int V = B * NR;
    constexpr int BM = ADJ_MASKED_B < B ? ADJ_MASKED_B : B;  // degrees per masked block
    static_assert(64 % V == 0 && V >= 8, "block values must divide the wave");
    __shared__ double red[V * 16];
    int m, chunk;
    xcd_map(nchunk, m, chunk);
    if (m > mmax)
        return;
    const int lane = threadIdx.x;
    const StartInfo si = st[m];
    const int l0 = si.l0;
    if (l0 > lmax || lfirst[m * nchunk + chunk] > lmax)
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
        rg[r] = ring_init<ADJ_IN_EXP>(si, q, ntheta, active, SPIN);
        ph[r] = slice_phase<SPIN>(rg[r]);
        double2 fpn = make_double2(0, 0), fps = fpn, fmn = fpn, fms = fpn;
        if (active) {
            const int jn = q, js = ntheta - 1 - q;
            const typename cplxk<T>::type *colp = D + (size_t)(SPIN ? m + mmax : m) * nd;
            fpn = ring_in<T>(colp, jn, ntheta, nd, ms);
            if (js != jn) {
                fps = ring_in<T>(colp, js, ntheta, nd, ms);
                fps.x *= sfix;
                fps.y *= sfix;
            }
            if (SPIN) {
                const typename cplxk<T>::type *colm = D + (size_t)(mmax - m) * nd;
                fmn = ring_in<T>(colm, jn, ntheta, nd, ms);
                if (js != jn) {
                    fms = ring_in<T>(colm, js, ntheta, nd, ms);
                    fms.x *= sfix;
                    fms.y *= sfix;
                }
            }
        }
        if (GRAD) {  // X_e, X_o, Y_e, Y_o (see adj_acc_grad)
            const double sg = (s & 1) ? -1.0 : 1.0;
            in[r].v[0] = fpn.x + sg * fms.x; in[r].v[1] = fpn.y - sg * fms.y;
            in[r].v[2] = fpn.x - sg * fms.x; in[r].v[3] = fpn.y + sg * fms.y;
            in[r].v[4] = fps.x + sg * fmn.x; in[r].v[5] = fps.y - sg * fmn.y;
            in[r].v[6] = -fps.x + sg * fmn.x; in[r].v[7] = -fps.y - sg * fmn.y;
        } else if (SPIN) {
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
    bool all_in = true, some_in = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        all_in = all_in && ph[r] == 2;
        some_in = some_in || ph[r] != 0;
    }

    // Reduce the block sums cb (VB values: VB / NR degrees) over the wave and add them
    // to acc (degrees lb..).
    auto reduce_add = [&](auto &cb, int lb) {
        constexpr int VB = std::extent<std::remove_reference_t<decltype(cb)>>::value;
        static_assert(64 % VB == 0 && VB >= 8 && VB <= V, "block values must divide the wave");
        // stage 1: lanes L, L + 32 -> VB/2 values; value k + (L / 32) VB/2 in slot k
        double c1[VB / 2];
#pragma unroll
        for (int k = 0; k < VB / 2; ++k)
            c1[k] = swap_add32(cb[k], cb[k + VB / 2]);
        // stage 2: rows (0,1), (2,3) -> VB/4 values per lane; slot k of row g holds
        // value k + (g & 1) VB/4 + (g >> 1) VB/2, partially summed over 4 lanes
        double c2[VB / 4];
#pragma unroll
        for (int k = 0; k < VB / 4; ++k)
            c2[k] = swap_add16(c1[k], c1[k + VB / 4]);
        const int g = lane >> 4, li = lane & 15;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < VB / 4; ++k) {
            const int vv = k + (g & 1) * (VB / 4) + (g >> 1) * (VB / 2);
            red[vv * 16 + ((li + vv) & 15)] = c2[k];
        }
        __syncthreads();
        constexpr int H = 64 / VB;      // lanes per value
        constexpr int SPAN = 16 / H;    // row partials summed per lane
        const int v = lane % VB, h = lane / VB;
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < SPAN; ++i)
            sum += red[v * 16 + ((h * SPAN + i + v) & 15)];
#pragma unroll
        for (int d = VB; d < 64; d <<= 1)
            sum += __shfl_xor(sum, d, 64);
        if (lane < VB && lb + lane / NR <= lmax)
            unsafeAtomicAdd(acc + (base + lb) * NR + lane, sum);
    };
    // per-lane sums of a block of BB = size / NC degrees -> the values reduced over
    // the wave
    auto reduce_block = [&](auto &cf, int lb) {
        constexpr int BB = std::extent<std::remove_reference_t<decltype(cf)>>::value / NC;
        if constexpr (GRAD) {
            double cr[2 * BB];
#pragma unroll
            for (int b = 0; b < BB; ++b) {
                cr[2 * b] = cf[4 * b] + cf[4 * b + 2];
                cr[2 * b + 1] = cf[4 * b + 1] + cf[4 * b + 3];
            }
            reduce_add(cr, lb);
        } else {
            reduce_add(cf, lb);
        }
    };
    // Masked block of BM degrees: channels out of range (offset < 0, constant inside a
    // block) get the weight 0 for the block; rescaling and phase update at its end.
    // Only partial blocks at the end (TAIL) check the degree bound.
    auto masked_block = [&](int lb, auto tail) {
        constexpr bool TAIL = decltype(tail)::value;
        double cb[BM * NC];
#pragma unroll
        for (int k = 0; k < BM * NC; ++k)
            cb[k] = 0.0;
        const double2 *abl = ab + base + lb;
        const bool had_some = some_in;
        double wa[R], wb[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            wa[r] = rg[r].ea == 0 ? 1.0 : 0.0;
            wb[r] = (SPIN && rg[r].eb == 0) ? 1.0 : 0.0;
        }
#pragma unroll
        for (int b = 0; b < BM; b += 2) {
            const int l = lb + b;
            if (TAIL && l > lmax)
                break;
            const double2 c0 = abl[b];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                adj_acc_any<SPIN, GRAD, 1>(cb + b * NC, in[r], rg[r].a1 * wa[r], rg[r].b1 * wb[r]);
                ring_advance<SPIN>(rg[r], c0.x, c0.y);
            }
            if (TAIL && l + 1 > lmax)
                break;
            const double2 c1 = abl[b + 1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                adj_acc_any<SPIN, GRAD, -1>(cb + (b + 1) * NC, in[r], rg[r].a1 * wa[r],
                                            rg[r].b1 * wb[r]);
                ring_advance<SPIN>(rg[r], c1.x, c1.y);
            }
            // one degree pair per scheduling region: hoisting later degrees'
            // recurrence steps ahead of this pair's sums costs registers
            __builtin_amdgcn_sched_barrier(0);
        }
        all_in = true;
        some_in = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ring_rescale<SPIN, ADJ_IN_EXP>(rg[r]);
            const int p = slice_phase<SPIN>(rg[r]);
            all_in = all_in && p == 2;
            some_in = some_in || p != 0;
        }
        if (had_some)  // otherwise every lane was out of range for the whole block
            reduce_block(cb, lb);
    };
    // Sequential loops (no loop-carried value crosses a branch merge): silent blocks
    // until some lane is in range, masked full blocks until every lane is, full plain
    // blocks, and masked partial blocks at the end.
    int lb = l0;
    silent_blocks<SPIN, ADJ_IN_EXP>(rg, ab + base, lb, lmax, all_in, some_in);
    for (; lb + BM - 1 <= lmax && !all_in; lb += BM)
        masked_block(lb, flag<false>());
    // Plain blocks; the coefficients of each degree pair are loaded one pair ahead
    // (across block ends too), so the scalar loads overlap the current pair's work.
    if (lb + B - 1 <= lmax) {
        double2 q0 = ab[base + lb], q1 = ab[base + lb + 1];
        for (; lb + B - 1 <= lmax; lb += B) {
            double cb[B * NC];
#pragma unroll
            for (int k = 0; k < B * NC; ++k)
                cb[k] = 0.0;
#pragma unroll
            for (int b = 0; b < B; b += 2) {
                const int ln = lb + b + 2;                    // next pair
                const int lc = ln + 1 <= lmax ? ln : lb + b;  // stays inside this m's table
                const double2 n0 = ab[base + lc], n1 = ab[base + lc + 1];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    adj_acc_any<SPIN, GRAD, 1>(cb + b * NC, in[r], rg[r].a1, rg[r].b1);
                    ring_advance<SPIN>(rg[r], q0.x, q0.y);
                    adj_acc_any<SPIN, GRAD, -1>(cb + (b + 1) * NC, in[r], rg[r].a1, rg[r].b1);
                    ring_advance<SPIN>(rg[r], q1.x, q1.y);
                }
                q0 = n0;
                q1 = n1;
            }
            reduce_block(cb, lb);
        }
    }
    for (; lb <= lmax; lb += BM)
        masked_block(lb, flag<true>());
}

template <int R, int B>
static void adj_launch(const gsht_plan &p, const void *Din, bool grad, hipStream_t s)
{
    dim3 blk(64), grd(xcd_grid(p.mmax, p.adj_nchunk));
#define GSHT_LEG_ADJ(T, SP, G, C)                                                                \
    hipLaunchKernelGGL((leg_adjoint_kernel<T, SP, R, B, G>), grd, blk, 0, s, p.leg.ab,           \
                       p.leg.start, p.leg.lfirst_adj, (const C *)Din, p.lmax, p.mmax, p.spin,     \
                       p.ntheta, p.nd, p.npairs, p.adj_nchunk, p.acc)
    if (p.prec == GSHT_F64) {
        if (p.spin && grad) GSHT_LEG_ADJ(double, true, true, double2);
        else if (p.spin) GSHT_LEG_ADJ(double, true, false, double2);
        else GSHT_LEG_ADJ(double, false, false, double2);
    } else {
        if (p.spin && grad) GSHT_LEG_ADJ(float, true, true, float2);
        else if (p.spin) GSHT_LEG_ADJ(float, true, false, float2);
        else GSHT_LEG_ADJ(float, false, false, float2);
    }
#undef GSHT_LEG_ADJ
}


hipError_t launch_leg_live_r1(const gsht_plan &p, int32_t *lfirst1, hipStream_t s)
{
    live_launch(p, 1, (p.npairs + 63) / 64, SYN_IN_EXP, lfirst1, s);
    return hipGetLastError();
}

hipError_t launch_zero(void *ptr, size_t bytes, hipStream_t s);

hipError_t launch_leg_adjoint(const gsht_plan &p, const void *Din, bool grad, hipStream_t s)
{
    hipError_t e = launch_zero(p.acc, sizeof(double) * (size_t)p.nalm * 2 * p.ncomp, s);
    if (e != hipSuccess)
        return e;
    const int key = p.adj_r * 100 + p.adj_b;
    switch (key) {
    case 108: adj_launch<1, 8>(p, Din, grad, s); break;
    case 208: adj_launch<2, 8>(p, Din, grad, s); break;
    case 204: adj_launch<2, 4>(p, Din, grad, s); break;
    case 404: adj_launch<4, 4>(p, Din, grad, s); break;
    case 308: adj_launch<3, 8>(p, Din, grad, s); break;
    case 304: adj_launch<3, 4>(p, Din, grad, s); break;
    case 408: adj_launch<4, 8>(p, Din, grad, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gsht

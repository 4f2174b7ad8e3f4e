// Matrix-core forms of the Legendre step for several maps sharing one geometry (FP32
// plans): the recurrence of legendre_kernels.hip in FP64, the degree sums as FP16
// split products on v_mfma_f32_32x32x16_f16 with FP32 accumulation.
#include "legendre_device.hpp"

namespace gsht {

// ---- several maps on the matrix cores (FP32 form) ------------------------------------

// For NM = 8 NCB maps sharing one geometry, the degree sums of one m are matrix
// products: per block of 16 degrees, the [64 ring pairs x 16 degrees] Legendre values
// of a channel times [16 degrees x 32 NCB] coefficient columns.  The recurrence runs
// in FP64 exactly as above (one slice of 64 ring pairs per wave); its values (|p_l| <=
// sqrt((2 l + 1) / 4 pi) / N_l, within FP16 range for lmax <= 8192) and the
// coefficients, scaled per (m, map) so that the largest lies in [2^7, 2^8), are split
// into FP16 pairs hi + lo (hi the value rounded towards zero, lo the remainder,
// likewise) and multiplied on the matrix cores (v_mfma_f32_32x32x16_f16) with FP32
// accumulation as hi hi + hi lo + lo hi; the dropped lo lo term and the split are
// below 2^-21 relative.  Values of a channel still carrying an exponent offset enter
// as 0.  Columns 4k..4k+3 of map k: channel +s ("a"): Re, Im of u+ (N+) and SG Re, Im
// u- (S-); channel -s ("b"): Re, Im u- (N-) and SG Re, Im u+ (S+); spin 0: u (N) and
// SG u (S), SG = (-1)^(l - l0).  Operand layouts of the 32x32x16 product: A row =
// lane % 32, B column = lane % 32, degree 8 (lane / 32) + j in element j of both;
// result element r of lane i is row 8 (r / 4) + 4 (i / 32) + r % 4, column i % 32.
// The loop is software-pipelined: the recurrence and conversion of block kb + 1 and
// the loads of its coefficient tiles are independent of block kb's products, so the
// vector and matrix units overlap.

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

constexpr int MK = 16;  // degrees per matrix step

// hi (x, y) rounded towards zero to FP16, lo the FP16 remainder
__device__ inline void split_pair(float x, float y, unsigned &hi, unsigned &lo)
{
    const half2_t h = __builtin_bit_cast(half2_t, __builtin_amdgcn_cvt_pkrtz(x, y));
    hi = __builtin_bit_cast(unsigned, h);
    lo = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(x - (float)h[0], y - (float)h[1]));
}

// Lane L holds degrees 0..7 of its ring in x and 8..15 in y.  Afterwards x is the A
// operand of ring pairs 0..31 (lanes 32..63 carrying degrees 8..15 of ring L - 32)
// and y that of ring pairs 32..63.
__device__ inline void to_operands(u32x4_t &x, u32x4_t &y)
{
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const auto r = __builtin_amdgcn_permlane32_swap(x[d], y[d], false, false);
        x[d] = r[0];
        y[d] = r[1];
    }
}

// rescale_channel without branches (selects only, so that the block's matrix
// products can be scheduled among the recurrence steps).  A fold happens only at
// e = -512 or -1024 (values reach at most 2^288 before the next check), where 2^e is
// still a double.
template <int INX>
__device__ inline void rescale_channel_sel(double &p0, double &p1, int &e)
{
    const bool neg = e < 0;
    const bool fold = neg && fabs(p1) >= ldexp(1.0, INX - e);
    const bool down = neg && !fold && fabs(p1) >= TWO_P256;
    const double f = fold ? ldexp(1.0, e) : (down ? TWO_M512 : 1.0);
    p0 *= f;
    p1 *= f;
    e = fold ? 0 : (down ? e + 512 : e);
}

// One channel's operands: [0] hi rings 0..31, [1] hi rings 32..63, [2], [3] lo.
struct AOps {
    u32x4_t v[4];
};

// Values of degrees lb .. lb + 15 of both channels as operands, advancing the
// recurrence by 16 degrees (coefficients past lmax read the zero entry at lmax).
template <bool SPIN>
__device__ inline void make_a(Ring &rg, const double2 *__restrict__ abm, int lb, int lmax,
                              AOps &A, AOps &B)
{
    const bool ia = rg.ea == 0, ib = SPIN && rg.eb == 0;
    float fa[MK], fb[MK];
#pragma unroll
    for (int j = 0; j < MK; ++j) {
        fa[j] = ia ? (float)rg.a1 : 0.f;
        fb[j] = ib ? (float)rg.b1 : 0.f;
        const int l = lb + j;
        const double2 c = abm[l < lmax ? l : lmax];
        ring_advance<SPIN>(rg, c.x, c.y);
    }
    rescale_channel_sel<SYN_IN_EXP>(rg.a0, rg.a1, rg.ea);
    if (SPIN)
        rescale_channel_sel<SYN_IN_EXP>(rg.b0, rg.b1, rg.eb);
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        unsigned hi, lo;
        split_pair(fa[2 * d], fa[2 * d + 1], hi, lo);
        A.v[d / 4][d % 4] = hi;
        A.v[2 + d / 4][d % 4] = lo;
        if (SPIN) {
            split_pair(fb[2 * d], fb[2 * d + 1], hi, lo);
            B.v[d / 4][d % 4] = hi;
            B.v[2 + d / 4][d % 4] = lo;
        }
    }
    to_operands(A.v[0], A.v[1]);
    to_operands(A.v[2], A.v[3]);
    if (SPIN) {
        to_operands(B.v[0], B.v[1]);
        to_operands(B.v[2], B.v[3]);
    }
}

__device__ inline f32x16_t mma(const u32x4_t &a, const u32x4_t &b, const f32x16_t &c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8_t, a),
                                                  __builtin_bit_cast(half8_t, b), c, 0, 0, 0);
}

// Coefficient tiles: per m, nkb(m) = ceil((lmax - l0 + 1) / 16) blocks starting at
// boff[m]; block kb holds [type][cb][hi, lo][lane] half8 entries for degrees
// l0 + 16 kb + 8 (lane / 32) + j.  oscale[m][map] undoes the coefficient scaling.
template <bool SPIN, int NCB>
__global__ __launch_bounds__(64) void leg_synth_mfma_kernel(
    const double2 *__restrict__ ab, const StartInfo *__restrict__ st,
    const int32_t *__restrict__ lfirst, const int64_t *__restrict__ boff,
    const u32x4_t *__restrict__ Bt, const float *__restrict__ oscale, int nm, int lmax, int mmax,
    int s, int ntheta, int nd, int npairs, int nchunk, size_t dstride, float2 *__restrict__ D)
{
    constexpr int NT = SPIN ? 2 : 1;
    constexpr int NMX = 8 * NCB;
    constexpr int BLK = NT * NCB * 2 * 64;  // 16-byte entries per block
    __shared__ float tile[64][33];
    int m, chunk;
    xcd_map(nchunk, m, chunk);
    if (m > mmax)
        return;
    const int lane = threadIdx.x;
    const StartInfo si = st[m];
    const int l0 = si.l0;
    const bool live = (l0 <= lmax) && (lfirst[m * nchunk + chunk] <= lmax);
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double2 *abm = ab + base;
    const int q = chunk * 64 + lane;
    Ring rg = ring_init<SYN_IN_EXP>(si, q, ntheta, live && q < npairs, SPIN);
    f32x16_t acc[2][NT][NCB];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int c = 0; c < NCB; ++c)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    acc[h][t][c][r] = 0.f;
    if (live) {
        const u32x4_t *bm = Bt + boff[m] * BLK + lane;
        const int nkb = (lmax - l0 + MK) / MK;
        int kb = 0;
        // blocks before any lane is in range: recurrence only
        while (kb < nkb && slice_phase<SPIN>(rg) == 0) {
#pragma unroll 4
            for (int j = 0; j < MK; ++j) {
                const int l = l0 + MK * kb + j;
                const double2 c = abm[l < lmax ? l : lmax];
                ring_advance<SPIN>(rg, c.x, c.y);
            }
            ring_rescale<SPIN, SYN_IN_EXP>(rg);
            ++kb;
        }
        if (kb < nkb) {
            AOps A[NT], An[NT];
            u32x4_t Bc[NT][NCB][2], Bn[NT][NCB][2];
            auto load_b = [&](int k, u32x4_t (&Bx)[NT][NCB][2]) {
                const u32x4_t *bb = bm + (int64_t)k * BLK;
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int c = 0; c < NCB; ++c)
#pragma unroll
                        for (int hl = 0; hl < 2; ++hl)
                            Bx[t][c][hl] = bb[((t * NCB + c) * 2 + hl) * 64];
            };
            load_b(kb, Bc);
            make_a<SPIN>(rg, abm, l0 + MK * kb, lmax, A[0], A[NT - 1]);
            for (; kb < nkb; ++kb) {
                // next block (past the end: a harmless repeat of the last tile and
                // recurrence steps on zero coefficients)
                load_b(kb + 1 < nkb ? kb + 1 : kb, Bn);
                make_a<SPIN>(rg, abm, l0 + MK * (kb + 1), lmax, An[0], An[NT - 1]);
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int c = 0; c < NCB; ++c)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            f32x16_t x = acc[h][t][c];
                            x = mma(A[t].v[h], Bc[t][c][0], x);
                            x = mma(A[t].v[h], Bc[t][c][1], x);
                            x = mma(A[t].v[2 + h], Bc[t][c][0], x);
                            acc[h][t][c] = x;
                        }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    A[t] = An[t];
#pragma unroll
                    for (int c = 0; c < NCB; ++c) {
                        Bc[t][c][0] = Bn[t][c][0];
                        Bc[t][c][1] = Bn[t][c][1];
                    }
                }
            }
        }
    }
    // Results through LDS, one (type, column block) at a time: lane L then holds the
    // 32 columns of ring pair L.
    const double sfix = ((l0 + m) & 1) ? -1.0 : 1.0;
    const double ms = ((s + m) & 1) ? -1.0 : 1.0;
    const int jn = q, js = ntheta - 1 - q;
    const int rbase = 4 * (lane / 32), col = lane % 32;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    tile[32 * h + 8 * (r / 4) + rbase + r % 4][col] = acc[h][t][c][r];
            __syncthreads();
            if (q < npairs) {
#pragma unroll 1
                for (int k = 0; k < 8; ++k) {
                    const int map = 8 * c + k;
                    if (map >= nm)
                        break;
                    const double f = oscale[m * NMX + map];
                    const double v0 = f * tile[lane][4 * k], v1 = f * tile[lane][4 * k + 1];
                    const double v2 = f * tile[lane][4 * k + 2], v3 = f * tile[lane][4 * k + 3];
                    float2 *Dk = D + (size_t)map * dstride;
                    if (!SPIN) {
                        float2 *colp = Dk + (size_t)m * nd;
                        put_ring<float>(colp, jn, ntheta, nd, ms, v0, v1);
                        if (js != jn)
                            put_ring<float>(colp, js, ntheta, nd, ms, sfix * v2, sfix * v3);
                    } else if (t == 0) {  // N+, S-
                        put_ring<float>(Dk + (size_t)(m + mmax) * nd, jn, ntheta, nd, ms, v0, v1);
                        if (m > 0 && js != jn)
                            put_ring<float>(Dk + (size_t)(mmax - m) * nd, js, ntheta, nd, ms,
                                            sfix * v2, sfix * v3);
                    } else {  // N-, S+
                        if (m > 0)
                            put_ring<float>(Dk + (size_t)(mmax - m) * nd, jn, ntheta, nd, ms, v0, v1);
                        if (js != jn)
                            put_ring<float>(Dk + (size_t)(m + mmax) * nd, js, ntheta, nd, ms,
                                            sfix * v2, sfix * v3);
                    }
                }
            }
            __syncthreads();
        }
}

hipError_t launch_leg_synth_mfma(const gsht_plan &p, int nm, const void *Bt, const float *oscale,
                                 const int64_t *boff, const int32_t *lfirst1, void *Dout,
                                 size_t dstride, hipStream_t s)
{
    if (p.prec != GSHT_F32 || nm < 1 || nm > 16)
        return hipErrorInvalidValue;
    const int nchunk = (p.npairs + 63) / 64;
    dim3 blk(64), grd(xcd_grid(p.mmax, nchunk));
#define GSHT_LEG_MFMA(SP, NCB)                                                                   \
    hipLaunchKernelGGL((leg_synth_mfma_kernel<SP, NCB>), grd, blk, 0, s, p.leg.ab, p.leg.start,  \
                       lfirst1, boff, (const u32x4_t *)Bt, oscale, nm, p.lmax, p.mmax, p.spin,    \
                       p.ntheta, p.nd, p.npairs, nchunk, dstride, (float2 *)Dout)
    if (p.spin) {
        if (nm > 8) GSHT_LEG_MFMA(true, 2);
        else GSHT_LEG_MFMA(true, 1);
    } else {
        if (nm > 8) GSHT_LEG_MFMA(false, 2);
        else GSHT_LEG_MFMA(false, 1);
    }
#undef GSHT_LEG_MFMA
    return hipGetLastError();
}

}  // namespace gsht

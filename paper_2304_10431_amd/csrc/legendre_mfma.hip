// Matrix-core forms of the Legendre step for several maps sharing one geometry (FP32
// plans): the recurrence of legendre_kernels.hip in FP64, the degree sums as FP16
// split products on v_mfma_f32_32x32x16_f16 with FP32 accumulation.
#include <algorithm>
#include <cstdlib>

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
    rescale_channel<SYN_IN_EXP>(rg.a0, rg.a1, rg.ea);
    if (SPIN)
        rescale_channel<SYN_IN_EXP>(rg.b0, rg.b1, rg.eb);
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
__global__ __launch_bounds__(64, 2) void leg_synth_mfma_kernel(
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
            auto products = [&](const AOps (&Ax)[NT], const u32x4_t (&Bx)[NT][NCB][2]) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int c = 0; c < NCB; ++c)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            f32x16_t x = acc[h][t][c];
                            x = mma(Ax[t].v[h], Bx[t][c][0], x);
                            x = mma(Ax[t].v[h], Bx[t][c][1], x);
                            x = mma(Ax[t].v[2 + h], Bx[t][c][0], x);
                            acc[h][t][c] = x;
                        }
            };
            load_b(kb, Bc);
            make_a<SPIN>(rg, abm, l0 + MK * kb, lmax, A[0], A[NT - 1]);
            // two blocks per iteration with the operand sets swapping roles, so no
            // register copies between blocks; the next block's operands (past the
            // end: a harmless repeat of the last tile and recurrence steps on zero
            // coefficients) are formed while the current block's products run
            for (; kb + 1 < nkb; kb += 2) {
                load_b(kb + 1, Bn);
                make_a<SPIN>(rg, abm, l0 + MK * (kb + 1), lmax, An[0], An[NT - 1]);
                products(A, Bc);
                load_b(kb + 2 < nkb ? kb + 2 : kb + 1, Bc);
                make_a<SPIN>(rg, abm, l0 + MK * (kb + 2), lmax, A[0], A[NT - 1]);
                products(An, Bn);
            }
            if (kb < nkb)
                products(A, Bc);
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

// ---- adjoint of several maps on the matrix cores (FP32 form) ------------------------

// The adjoint sums of one m are products over ring pairs: for a block of 16 degrees,
// C_t[column][degree] = sum_q F_t[q][column] p_t,l(q) with the per-ring inputs F
// (columns per map: channel +s: Re, Im F+(N), Re, Im conj F-(S'); channel -s: Re, Im
// conj F-(N), Re, Im F+(S'); spin 0: Re, Im F(N), Re, Im F(S'), S' the south ring
// times (-1)^(l0+m), exactly the inputs of leg_adjoint_kernel) and then
//   S+ = C_a[F+(N)] + SG C_b[F+(S')],  S- = C_b[conj F-(N)] + SG C_a[conj F-(S')],
//   spin 0: b = C[F(N)] + SG C[F(S')],  SG = (-1)^(l - l0).
// One workgroup per m; its W waves split the ring slices (64 pairs each, S slices per
// wave, recurrence state in registers, FP64, threshold 2^-256 as the FP64 adjoint).
// Per block a wave writes the FP16 hi/lo parts of its slice's Legendre values to an
// LDS slab [hi, lo][16 degrees][64 rings (+4 pad)] as (channel +s, channel -s) pairs,
// reads them back in the B layout of v_mfma_f32_16x16x32_f16 (degree = lane % 16,
// rings 8 (lane / 16) + j of a 32-ring step) and multiplies the F tiles (A layout:
// column = lane % 16, same rings), hi hi + hi lo + lo hi.  The W partial results of a
// block are summed through LDS (the slabs' space) and written once, so the output
// needs no atomics.  Result element r of lane i is column 4 (i / 16) + r (map
// 4 cb + i / 16, entry r), degree i % 16.

typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int AK = 16;    // degrees per block
constexpr int PROW = 68;  // LDS slab row: 64 rings + 4 words of padding

__device__ inline f32x4_t mma16(const u32x4_t &a, const u32x4_t &b, const f32x4_t &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8_t, a),
                                                  __builtin_bit_cast(half8_t, b), c, 0, 0, 0);
}

// low (SEL 0) or high (SEL 1) FP16 halves of two words, packed
template <int SEL>
__device__ inline unsigned halves(unsigned x, unsigned y)
{
    return SEL == 0 ? __builtin_amdgcn_perm(y, x, 0x05040100u) : __builtin_amdgcn_perm(y, x, 0x07060302u);
}

// The eight per-ring adjoint inputs of ring pair q from one map's doubled columns.
__device__ inline void adj_inputs(const float2 *__restrict__ D, int m, int mmax, int spin, int q,
                                  int ntheta, int nd, int npairs, float (&v)[8])
{
#pragma unroll
    for (int k = 0; k < 8; ++k)
        v[k] = 0.f;
    if (q >= npairs)
        return;
    const double ms = ((spin + m) & 1) ? -1.0 : 1.0;
    const int l0 = m > spin ? m : spin;
    const double sfix = ((l0 + m) & 1) ? -1.0 : 1.0;
    const int jn = q, js = ntheta - 1 - q;
    const float2 *colp = D + (size_t)(spin ? m + mmax : m) * nd;
    double2 n = ring_in<float>(colp, jn, ntheta, nd, ms), so = make_double2(0.0, 0.0);
    if (js != jn) {
        so = ring_in<float>(colp, js, ntheta, nd, ms);
        so.x *= sfix;
        so.y *= sfix;
    }
    v[0] = (float)n.x; v[1] = (float)n.y; v[2] = (float)so.x; v[3] = (float)so.y;
    if (spin) {
        const float2 *colm = D + (size_t)(mmax - m) * nd;
        double2 mn = ring_in<float>(colm, jn, ntheta, nd, ms), msn = make_double2(0.0, 0.0);
        if (js != jn) {
            msn = ring_in<float>(colm, js, ntheta, nd, ms);
            msn.x *= sfix;
            msn.y *= sfix;
        }
        v[4] = (float)mn.x; v[5] = (float)-mn.y; v[6] = (float)msn.x; v[7] = (float)-msn.y;
    }
}

// F tiles: per (m, slice, 32-ring step ks) [type][cb][hi, lo][lane] half8 entries,
// column lane % 16 (map 4 cb + (lane % 16) / 4, entry lane % 4), ring pairs
// 64 slice + 32 ks + 8 (lane / 16) + j; per (m, map) scale 2^e (largest scaled input in
// [2^7, 2^8)), oscale[m][map] = 2^-e.  One workgroup per m.
template <int NCB>
__global__ __launch_bounds__(256) void prep_adj_mfma_kernel(
    const float2 *__restrict__ D, size_t dstride, int mmax, int spin, int ntheta, int nd,
    int npairs, int nslice, int nm, u32x4_t *__restrict__ At, float *__restrict__ oscale)
{
    constexpr int NMX = 4 * NCB;
    const int m = blockIdx.x, tid = threadIdx.x;
    const int nt = spin ? 2 : 1;
    const int tmap = tid / 16, tq = tid % 16;
    __shared__ unsigned mx[NMX];
    __shared__ float sc[NMX];
    __shared__ float V[NMX][8][33];
    if (tid < NMX)
        mx[tid] = 0u;
    __syncthreads();
    if (tmap < nm) {
        float lm = 0.f;
        for (int q = tq; q < npairs; q += 16) {
            float v[8];
            adj_inputs(D + (size_t)tmap * dstride, m, mmax, spin, q, ntheta, nd, npairs, v);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                lm = fmaxf(lm, fabsf(v[k]));
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
        sc[tid] = ldexpf(1.f, e);
        oscale[m * NMX + tid] = ldexpf(1.f, -e);
    }
    __syncthreads();
    const int per = nt * NCB * 2 * 64;
    for (int step = 0; step < 2 * nslice; ++step) {
        const int qb = 32 * step;
        if (tmap < NMX) {
            for (int h = 0; h < 2; ++h) {
                float v[8];
                adj_inputs(D + (size_t)(tmap < nm ? tmap : 0) * dstride, m, mmax, spin,
                           tmap < nm ? qb + tq + 16 * h : npairs, ntheta, nd, npairs, v);
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    V[tmap][k][tq + 16 * h] = v[k] * sc[tmap];
            }
        }
        __syncthreads();
        for (int idx = tid; idx < per; idx += blockDim.x) {
            const int lane = idx % 64, hl = (idx / 64) % 2, cb = (idx / 128) % NCB;
            const int t = idx / (128 * NCB);
            const int col = lane % 16, map = 4 * cb + col / 4, e = col % 4;
            // entry e of type t -> input index
            const int src = spin == 0 ? e : (t == 0 ? (e < 2 ? e : e + 4) : (e < 2 ? e + 4 : e));
            half8_t v;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float f = V[map][src][8 * (lane / 16) + j];
                const auto hp = __builtin_amdgcn_cvt_pkrtz(f, 0.f);
                v[j] = hl == 0 ? hp[0] : __builtin_amdgcn_cvt_pkrtz(f - (float)hp[0], 0.f)[0];
            }
            At[((int64_t)m * 2 * nslice + step) * per + idx] = __builtin_bit_cast(u32x4_t, v);
        }
        __syncthreads();
    }
}

// Most waves per workgroup with NB sub-blocks (the slabs fill the LDS budget): the
// launch bound, so that the compiler may give each wave the registers that leaves.
template <int NB>
constexpr int adj_wmax()
{
    return (int)(COL_MAX_BYTES / (2 * AK * NB * PROW * 4)) < 16 ? (int)(COL_MAX_BYTES / (2 * AK * NB * PROW * 4)) : 16;
}

// Recurrence state of every ring of one m between blocks, structure of arrays over
// n = 64 nslice rings: x, a0, a1, b0, b1 (double), then ea, eb (int).
constexpr size_t RS_BYTES = 5 * sizeof(double) + 2 * sizeof(int);  // per ring

__device__ inline void ring_load(Ring &r, const unsigned char *rs, int n, int idx)
{
    const double *d = reinterpret_cast<const double *>(rs);
    const int *e = reinterpret_cast<const int *>(d + 5 * (size_t)n);
    r.x = d[idx];
    r.a0 = d[n + idx];
    r.a1 = d[2 * n + idx];
    r.b0 = d[3 * n + idx];
    r.b1 = d[4 * n + idx];
    r.ea = e[idx];
    r.eb = e[n + idx];
}

__device__ inline void ring_store(const Ring &r, unsigned char *rs, int n, int idx)
{
    double *d = reinterpret_cast<double *>(rs);
    int *e = reinterpret_cast<int *>(d + 5 * (size_t)n);
    d[idx] = r.x;
    d[n + idx] = r.a0;
    d[2 * n + idx] = r.a1;
    d[3 * n + idx] = r.b0;
    d[4 * n + idx] = r.b1;
    e[idx] = r.ea;
    e[n + idx] = r.eb;
}

template <bool SPIN, int NCB, int NB>
__global__ __launch_bounds__(64 * adj_wmax<NB>()) void leg_adjoint_mfma_kernel(
    const double2 *__restrict__ ab, const StartInfo *__restrict__ st,
    const int32_t *__restrict__ lfirst, const u32x4_t *__restrict__ At,
    const float *__restrict__ oscale, int nm, int lmax, int mmax, int ntheta, int npairs,
    int nslice, int64_t nalm, unsigned char *__restrict__ rstate, double *__restrict__ accm)
{
    constexpr int NT = SPIN ? 2 : 1;
    constexpr int NR = SPIN ? 4 : 2;
    constexpr int NMX = 4 * NCB;
    constexpr int PER = NT * NCB * 2 * 64;  // tile entries per 32-ring step
    constexpr int BK = AK * NB;             // degrees per block
    extern __shared__ unsigned smem[];
    const int W = blockDim.x / 64;
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int m = blockIdx.x;
    if (m > mmax)
        return;
    const StartInfo si = st[m];
    const int l0 = si.l0;
    if (l0 > lmax)
        return;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double2 *abm = ab + base;
    unsigned *slab = smem + w * (2 * BK * PROW);
    f32x4_t *red = reinterpret_cast<f32x4_t *>(smem);  // [W][NB][NT][NCB][64], after a barrier
    const int nr = 64 * nslice;
    unsigned char *rs = rstate + (size_t)m * nr * RS_BYTES;
    // slices of this wave: w, w + W, ...; live ones in a bit mask
    unsigned live = 0;
    for (int i = 0, sl = w; sl < nslice; ++i, sl += W) {
        const bool act = lfirst[m * nslice + sl] <= lmax;
        live |= act ? (1u << i) : 0u;
        const int q = 64 * sl + lane;
        const Ring r0 = ring_init<ADJ_IN_EXP>(si, q, ntheta, act && q < npairs, SPIN);
        ring_store(r0, rs, nr, q);
    }
    const int n = lane % 16, g = lane / 16;
    for (int lb = l0; lb <= lmax; lb += BK) {
        f32x4_t acc[NB][NT][NCB];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int c = 0; c < NCB; ++c)
                    acc[b][t][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
        for (int i = 0, sl = w; sl < nslice; ++i, sl += W) {
            if (!((live >> i) & 1u))
                continue;
            const int q = 64 * sl + lane;
            Ring rg;
            ring_load(rg, rs, nr, q);
            if (slice_phase<SPIN>(rg) == 0) {  // nothing in range: recurrence only
#pragma unroll 4
                for (int j = 0; j < BK; ++j) {
                    const int l = lb + j;
                    const double2 c = abm[l < lmax ? l : lmax];
                    ring_advance<SPIN>(rg, c.x, c.y);
                }
                rescale_channel<ADJ_IN_EXP>(rg.a0, rg.a1, rg.ea);
                if (SPIN)
                    rescale_channel<ADJ_IN_EXP>(rg.b0, rg.b1, rg.eb);
                ring_store(rg, rs, nr, q);
                continue;
            }
            // F tiles of both 32-ring steps, requested before the recurrence runs
            const u32x4_t *ap = At + ((int64_t)m * 2 * nslice + 2 * sl) * PER + lane;
            u32x4_t ah[2][NT][NCB], al[2][NT][NCB];
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int c = 0; c < NCB; ++c) {
                        ah[ks][t][c] = ap[ks * PER + ((t * NCB + c) * 2 + 0) * 64];
                        al[ks][t][c] = ap[ks * PER + ((t * NCB + c) * 2 + 1) * 64];
                    }
            // Legendre values of degrees lb .. lb + BK - 1 -> slab (hi, lo planes)
            const bool ia = rg.ea == 0, ib = SPIN && rg.eb == 0;
#pragma unroll 4
            for (int j = 0; j < BK; ++j) {
                const float fa = ia ? (float)rg.a1 : 0.f;
                const float fb = ib ? (float)rg.b1 : 0.f;
                const half2_t h = __builtin_bit_cast(half2_t, __builtin_amdgcn_cvt_pkrtz(fa, fb));
                const auto lo = __builtin_amdgcn_cvt_pkrtz(fa - (float)h[0], fb - (float)h[1]);
                slab[j * PROW + lane] = __builtin_bit_cast(unsigned, h);
                slab[(BK + j) * PROW + lane] = __builtin_bit_cast(unsigned, lo);
                const int l = lb + j;
                const double2 c = abm[l < lmax ? l : lmax];
                ring_advance<SPIN>(rg, c.x, c.y);
            }
            rescale_channel<ADJ_IN_EXP>(rg.a0, rg.a1, rg.ea);
            if (SPIN)
                rescale_channel<ADJ_IN_EXP>(rg.b0, rg.b1, rg.eb);
            ring_store(rg, rs, nr, q);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    // B operands: degree 16 b + n, ring pairs 32 ks + 8 g + j, both channels
                    const unsigned *ph = slab + (AK * b + n) * PROW + 32 * ks + 8 * g;
                    const unsigned *pl = ph + BK * PROW;
                    const u32x4_t h0 = *reinterpret_cast<const u32x4_t *>(ph);
                    const u32x4_t h1 = *reinterpret_cast<const u32x4_t *>(ph + 4);
                    const u32x4_t q0 = *reinterpret_cast<const u32x4_t *>(pl);
                    const u32x4_t q1 = *reinterpret_cast<const u32x4_t *>(pl + 4);
                    u32x4_t bh[NT], bl[NT];
                    bh[0] = u32x4_t{halves<0>(h0[0], h0[1]), halves<0>(h0[2], h0[3]),
                                    halves<0>(h1[0], h1[1]), halves<0>(h1[2], h1[3])};
                    bl[0] = u32x4_t{halves<0>(q0[0], q0[1]), halves<0>(q0[2], q0[3]),
                                    halves<0>(q1[0], q1[1]), halves<0>(q1[2], q1[3])};
                    if (SPIN) {
                        bh[NT - 1] = u32x4_t{halves<1>(h0[0], h0[1]), halves<1>(h0[2], h0[3]),
                                             halves<1>(h1[0], h1[1]), halves<1>(h1[2], h1[3])};
                        bl[NT - 1] = u32x4_t{halves<1>(q0[0], q0[1]), halves<1>(q0[2], q0[3]),
                                             halves<1>(q1[0], q1[1]), halves<1>(q1[2], q1[3])};
                    }
#pragma unroll
                    for (int t = 0; t < NT; ++t)
#pragma unroll
                        for (int c = 0; c < NCB; ++c) {
                            f32x4_t x = acc[b][t][c];
                            x = mma16(ah[ks][t][c], bh[t], x);
                            x = mma16(ah[ks][t][c], bl[t], x);
                            x = mma16(al[ks][t][c], bh[t], x);
                            acc[b][t][c] = x;
                        }
                }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // sum the waves' partial products and write the block's coefficients
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int c = 0; c < NCB; ++c)
                    red[(((w * NB + b) * NT + t) * NCB + c) * 64 + lane] = acc[b][t][c];
        __syncthreads();
        for (int o = threadIdx.x; o < NB * NCB * 64; o += blockDim.x) {
            const int b = o / (NCB * 64), c = (o / 64) % NCB, ln = o % 64;
            const int map = 4 * c + ln / 16, deg = AK * b + ln % 16;
            const int l = lb + deg;
            if (map >= nm || l > lmax)
                continue;
            f32x4_t A = f32x4_t{0.f, 0.f, 0.f, 0.f}, B = A;
            for (int ww = 0; ww < W; ++ww) {
                A += red[(((ww * NB + b) * NT + 0) * NCB + c) * 64 + ln];
                if (SPIN)
                    B += red[(((ww * NB + b) * NT + NT - 1) * NCB + c) * 64 + ln];
            }
            const double f = oscale[m * NMX + map];
            const double sg = ((l - l0) & 1) ? -1.0 : 1.0;
            double *out = accm + (int64_t)map * nalm * NR + (base + l) * NR;
            if (SPIN) {
                out[0] = f * ((double)A[0] + sg * (double)B[2]);
                out[1] = f * ((double)A[1] + sg * (double)B[3]);
                out[2] = f * ((double)B[0] + sg * (double)A[2]);
                out[3] = f * ((double)B[1] + sg * (double)A[3]);
            } else {
                out[0] = f * ((double)A[0] + sg * (double)A[2]);
                out[1] = f * ((double)A[1] + sg * (double)A[3]);
            }
        }
        __syncthreads();
    }
}

// Launch shape of the adjoint kernel: NB sub-blocks of 16 degrees per block (the F
// tiles of a slice serve all of them), W waves per workgroup within the LDS (slabs of
// 2 x 16 NB x 68 words each), at most 32 slices per wave (the live mask); W = 0 if
// the plan has more ring slices than that.  GSHT_ADJ_NB (1, 2 or 4) selects NB.
static int adj_nb()
{
    const char *e = getenv("GSHT_ADJ_NB");
    const int v = e ? atoi(e) : 4;
    return (v == 1 || v == 2) ? v : 4;
}

size_t adj_mfma_lds(int W, int NB) { return (size_t)W * 2 * AK * NB * PROW * 4; }

void adj_mfma_shape(const gsht_plan &p, int &S, int &W)
{
    const int nb = adj_nb();
    const int nslice = (p.npairs + 63) / 64;
    const int wmax = nb == 1 ? adj_wmax<1>() : nb == 2 ? adj_wmax<2>() : adj_wmax<4>();
    S = (nslice + wmax - 1) / wmax;
    W = (nslice + S - 1) / S;
    if (S > 32)
        S = W = 0;
}

size_t adj_mfma_state_bytes(const gsht_plan &p)
{
    return (size_t)(p.mmax + 1) * 64 * ((p.npairs + 63) / 64) * RS_BYTES;
}

hipError_t launch_prep_adj_mfma(const gsht_plan &p, int nm, const void *Din, size_t dstride,
                                void *tiles, float *oscale, hipStream_t s)
{
    if (p.prec != GSHT_F32 || nm < 1 || nm > 16)
        return hipErrorInvalidValue;
    const int nslice = (p.npairs + 63) / 64;
    dim3 blk(256), grd(p.mmax + 1);
    if (nm > 8)
        hipLaunchKernelGGL(prep_adj_mfma_kernel<4>, grd, blk, 0, s, (const float2 *)Din, dstride,
                           p.mmax, p.spin, p.ntheta, p.nd, p.npairs, nslice, nm, (u32x4_t *)tiles,
                           oscale);
    else
        hipLaunchKernelGGL(prep_adj_mfma_kernel<2>, grd, blk, 0, s, (const float2 *)Din, dstride,
                           p.mmax, p.spin, p.ntheta, p.nd, p.npairs, nslice, nm, (u32x4_t *)tiles,
                           oscale);
    return hipGetLastError();
}

template <bool SP, int NCB, int NB>
static hipError_t adj_mfma_go(const gsht_plan &p, int nm, int W, const void *tiles,
                              const float *oscale, const int32_t *lfirst1, void *rstate,
                              double *accm, hipStream_t s)
{
    const size_t lds = adj_mfma_lds(W, NB);
    hipError_t e = hipFuncSetAttribute((const void *)leg_adjoint_mfma_kernel<SP, NCB, NB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((leg_adjoint_mfma_kernel<SP, NCB, NB>), dim3(p.mmax + 1), dim3(64 * W), lds,
                       s, p.leg.ab, p.leg.start, lfirst1, (const u32x4_t *)tiles, oscale, nm,
                       p.lmax, p.mmax, p.ntheta, p.npairs, (p.npairs + 63) / 64, p.nalm,
                       (unsigned char *)rstate, accm);
    return hipGetLastError();
}

template <bool SP, int NCB>
static hipError_t adj_mfma_nb(const gsht_plan &p, int nm, int W, const void *tiles,
                              const float *oscale, const int32_t *lfirst1, void *rstate,
                              double *accm, hipStream_t s)
{
    switch (adj_nb()) {
    case 1: return adj_mfma_go<SP, NCB, 1>(p, nm, W, tiles, oscale, lfirst1, rstate, accm, s);
    case 2: return adj_mfma_go<SP, NCB, 2>(p, nm, W, tiles, oscale, lfirst1, rstate, accm, s);
    default: return adj_mfma_go<SP, NCB, 4>(p, nm, W, tiles, oscale, lfirst1, rstate, accm, s);
    }
}

hipError_t launch_leg_adjoint_mfma(const gsht_plan &p, int nm, const void *tiles,
                                   const float *oscale, const int32_t *lfirst1, void *rstate,
                                   double *accm, hipStream_t s)
{
    int S, W;
    adj_mfma_shape(p, S, W);
    if (p.prec != GSHT_F32 || nm < 1 || nm > 16 || W == 0)
        return hipErrorInvalidValue;
    if (p.spin)
        return nm > 8 ? adj_mfma_nb<true, 4>(p, nm, W, tiles, oscale, lfirst1, rstate, accm, s)
                      : adj_mfma_nb<true, 2>(p, nm, W, tiles, oscale, lfirst1, rstate, accm, s);
    return nm > 8 ? adj_mfma_nb<false, 4>(p, nm, W, tiles, oscale, lfirst1, rstate, accm, s)
                  : adj_mfma_nb<false, 2>(p, nm, W, tiles, oscale, lfirst1, rstate, accm, s);
}

}  // namespace gsht

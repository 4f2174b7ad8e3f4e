// Per-column FFT stage of the general SHT on gfx950 (Sect. 3: the FFT of the
// doubled meridians, the deconvolution / zero padding of the NUFFT, and the
// oversampled theta transform), with one workgroup per column and the column held
// in LDS, so that each column crosses HBM once on the way in and once on the way out.
//
//   forward:  D[col][0..nd)  --FFT_nd(-)-->  D^  --f(k,m), zero pad-->  E^[0..n1)
//             --FFT_n1(+)-->  E[col][a]   (only the torus rows the grid keeps)
//   adjoint:  E[col][kept rows]  --FFT_n1(-)-->  E^  --f(k,m)-->  D^[0..nd)
//             --FFT_nd(+)-->  D[col]
//
// f(k, m) = kfac1[|k|] kfac2[|m|] for |k| <= lmax and 0 otherwise, the same real
// factors both ways, so the adjoint stays the exact transpose of the forward.
// When n1 does not fit in LDS (FP64 at large n1) only the nd transform and the
// deconvolution are fused here and the theta transform runs separately on E.
//
// The FFTs are in-place mixed-radix decimation-in-frequency passes over LDS (radices
// 16, 8, 4, 2, 3, 5, 7): pass i splits sub-transforms of length L into radix r_i
// butterflies of stride s = L / r_i, each followed by the twiddles w_L^(q j).  The
// result sits in digit-reversed order; a host-built table gives the LDS position of
// every frequency.  Twiddles come from an FP64 table of w_n^k (one read per
// butterfly) and FP64 powers of it.
#include <algorithm>

#include "gsht_internal.hpp"

namespace gsht {

namespace {

constexpr int COL_THREADS = 1024;

template <typename T> struct cx;
template <> struct cx<float> { using type = float2; };
template <> struct cx<double> { using type = double2; };

// Values per thread when a whole column (at most COL_MAX_BYTES) is staged in
// registers between reading and overwriting the LDS buffer.
template <typename T>
constexpr int col_maxv()
{
    return (int)(COL_MAX_BYTES / sizeof(typename cx<T>::type)) / COL_THREADS;
}

template <typename C>
__device__ inline C cadd(C a, C b) { a.x += b.x; a.y += b.y; return a; }
template <typename C>
__device__ inline C csub(C a, C b) { a.x -= b.x; a.y -= b.y; return a; }

// ---- small DFTs in registers (DIR = -1 forward e^{-2 pi i}, +1 backward) ------

// cos, sin of 2 pi k / 16 for k < 8
__device__ constexpr double C16[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                                      0.38268343236508977173, 0.0, -0.38268343236508977173,
                                      -0.70710678118654752440, -0.92387953251128675613};
__device__ constexpr double S16[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440,
                                      0.92387953251128675613, 1.0, 0.92387953251128675613,
                                      0.70710678118654752440, 0.38268343236508977173};

// b * w_16^(DIR * idx) with w_16 = e^{2 pi i / 16}; idx is a compile-time constant
// after unrolling, so the trivial factors cost nothing.
template <typename C, int DIR>
__device__ inline C tw16(C b, int idx)
{
    using T = decltype(b.x);
    if (idx == 0)
        return b;
    C o;
    if (idx == 4) {  // multiply by DIR * i
        o.x = -DIR * b.y;
        o.y = DIR * b.x;
        return o;
    }
    const T c = (T)C16[idx], s = (T)(DIR * S16[idx]);
    o.x = b.x * c - b.y * s;
    o.y = b.x * s + b.y * c;
    return o;
}

template <int R>
__device__ constexpr int bitrev(int i)
{
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

// Radix-2 decimation in time over R <= 16 values (bit-reversed load, natural output).
template <typename C, int R, int DIR>
__device__ inline void dft_pow2(C (&v)[R])
{
    C w[R];
#pragma unroll
    for (int i = 0; i < R; ++i)
        w[bitrev<R>(i)] = v[i];
#pragma unroll
    for (int m = 2; m <= R; m <<= 1)
#pragma unroll
        for (int k0 = 0; k0 < R; k0 += m)
#pragma unroll
            for (int j = 0; j < m / 2; ++j) {
                const C a = w[k0 + j];
                const C b = tw16<C, DIR>(w[k0 + j + m / 2], j * (16 / m));
                w[k0 + j] = cadd(a, b);
                w[k0 + j + m / 2] = csub(a, b);
            }
#pragma unroll
    for (int i = 0; i < R; ++i)
        v[i] = w[i];
}

template <int R> struct OddTab;
template <> struct OddTab<3> {
    static constexpr double c[3] = {1.0, -0.5, -0.5};
    static constexpr double s[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
};
template <> struct OddTab<5> {
    static constexpr double c[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410,
                                    -0.80901699437494742410, 0.30901699437494742410};
    static constexpr double s[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917,
                                    -0.58778525229247312917, -0.95105651629515357212};
};
template <> struct OddTab<7> {
    static constexpr double c[7] = {1.0, 0.62348980185873353053, -0.22252093395631440429,
                                    -0.90096886790241912624, -0.90096886790241912624,
                                    -0.22252093395631440429, 0.62348980185873353053};
    static constexpr double s[7] = {0.0, 0.78183148246802980871, 0.97492791218182360702,
                                    0.43388373911755812048, -0.43388373911755812048,
                                    -0.97492791218182360702, -0.78183148246802980871};
};

// Odd prime R: X_q = v0 + sum_t [(v_t + v_{R-t}) cos(2 pi t q / R)
//                                 + DIR i (v_t - v_{R-t}) sin(2 pi t q / R)].
template <typename C, int R, int DIR>
__device__ inline void dft_odd(C (&v)[R])
{
    using T = decltype(v[0].x);
    constexpr int H = (R - 1) / 2;
    C sp[H], sm[H];
#pragma unroll
    for (int t = 1; t <= H; ++t) {
        sp[t - 1] = cadd(v[t], v[R - t]);
        sm[t - 1] = csub(v[t], v[R - t]);
    }
    C y[R];
    y[0] = v[0];
#pragma unroll
    for (int t = 0; t < H; ++t)
        y[0] = cadd(y[0], sp[t]);
#pragma unroll
    for (int q = 1; q <= H; ++q) {
        C a = v[0], b;
        b.x = 0;
        b.y = 0;
#pragma unroll
        for (int t = 1; t <= H; ++t) {
            const int k = (t * q) % R;
            const T c = (T)OddTab<R>::c[k], s = (T)OddTab<R>::s[k];
            a.x += c * sp[t - 1].x;
            a.y += c * sp[t - 1].y;
            b.x += s * sm[t - 1].x;
            b.y += s * sm[t - 1].y;
        }
        // X_q = a + DIR i b,  X_{R-q} = a - DIR i b
        y[q].x = a.x - DIR * b.y;
        y[q].y = a.y + DIR * b.x;
        y[R - q].x = a.x + DIR * b.y;
        y[R - q].y = a.y - DIR * b.x;
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
        v[i] = y[i];
}

template <typename C, int R, int DIR>
__device__ inline void dft(C (&v)[R])
{
    if constexpr ((R & (R - 1)) == 0)
        dft_pow2<C, R, DIR>(v);
    else
        dft_odd<C, R, DIR>(v);
}

// One decimation-in-frequency pass: butterflies b < n / R over sub-transforms of
// length L = R s; butterfly (sub, j) reads positions sub L + j + t s, t < R.
template <typename C, int R, int DIR>
__device__ inline void dif_pass(C *X, const double2 *__restrict__ tw, int n, int s)
{
    using T = decltype(X[0].x);
    const int L = R * s, tstep = n / L, nb = n / R;
    for (int b = threadIdx.x; b < nb; b += COL_THREADS) {
        const int sub = b / s, j = b - sub * s;
        const int base = sub * L + j;
        C v[R];
#pragma unroll
        for (int t = 0; t < R; ++t)
            v[t] = X[base + t * s];
        dft<C, R, DIR>(v);
        if (j != 0) {
            // w_L^(DIR q j) = (w_n^(tstep j))^q, powers formed in FP64
            double2 w1 = tw[tstep * j];
            if (DIR > 0)
                w1.y = -w1.y;
            double2 w = w1;
#pragma unroll
            for (int q = 1; q < R; ++q) {
                const T wr = (T)w.x, wi = (T)w.y;
                const C a = v[q];
                v[q].x = a.x * wr - a.y * wi;
                v[q].y = a.x * wi + a.y * wr;
                const double xr = w.x * w1.x - w.y * w1.y;
                w.y = w.x * w1.y + w.y * w1.x;
                w.x = xr;
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t)
            X[base + t * s] = v[t];
    }
}

// Whole transform in LDS (the block must hold the column before the call; the
// result is in digit-reversed order when it returns, after a barrier).
template <typename C, int DIR>
__device__ void lds_fft(C *X, const ColFFT &f)
{
    int L = f.n;
    for (int p = 0; p < f.npass; ++p) {
        const int r = f.radix[p];
        const int s = L / r;
        switch (r) {
        case 16: dif_pass<C, 16, DIR>(X, f.tw, f.n, s); break;
        case 8: dif_pass<C, 8, DIR>(X, f.tw, f.n, s); break;
        case 4: dif_pass<C, 4, DIR>(X, f.tw, f.n, s); break;
        case 2: dif_pass<C, 2, DIR>(X, f.tw, f.n, s); break;
        case 3: dif_pass<C, 3, DIR>(X, f.tw, f.n, s); break;
        case 5: dif_pass<C, 5, DIR>(X, f.tw, f.n, s); break;
        case 7: dif_pass<C, 7, DIR>(X, f.tw, f.n, s); break;
        default: break;
        }
        L = s;
        __syncthreads();
    }
}

__device__ inline bool row_kept(int a, int n1, int nrows, int a_min)
{
    int r = a - a_min;
    if (r >= n1)
        r -= n1;
    return r < nrows;  // a_min <= 0 and a < n1, so r >= 0
}

template <typename C>
__device__ inline C scale_c(C v, double f)
{
    using T = decltype(v.x);
    v.x = (T)(f * (double)v.x);
    v.y = (T)(f * (double)v.y);
    return v;
}

struct ColArgs {
    const double *kf1, *kf2;
    int lmax, mmax, spin, nd, n1, nrows, a_min;
};

__device__ inline int col_m(const ColArgs &a, int col) { return a.spin ? col - a.mmax : col; }

// FULL: D column -> E column (kept rows).  Otherwise D column -> zero-padded,
// deconvolved spectrum E^ over all n1 entries (the theta transform follows).
template <typename T, bool FULL>
__global__ __launch_bounds__(COL_THREADS) void column_fwd_kernel(
    const typename cx<T>::type *__restrict__ D, typename cx<T>::type *__restrict__ E, ColArgs a,
    ColFFT fd, ColFFT f1)
{
    using C = typename cx<T>::type;
    extern __shared__ unsigned char smem_raw[];
    C *X = reinterpret_cast<C *>(smem_raw);
    const int col = blockIdx.x, tid = threadIdx.x;
    const int m = col_m(a, col);
    const double fm = a.kf2[m < 0 ? -m : m];
    const C *dc = D + (size_t)col * a.nd;
    C *ec = E + (size_t)col * a.n1;
    for (int i = tid; i < a.nd; i += COL_THREADS)
        X[i] = dc[i];
    __syncthreads();
    lds_fft<C, -1>(X, fd);
    // deconvolution and zero padding: output i in [0, n1) <- frequency k
    auto deconv = [&](int i) {
        C o;
        o.x = 0;
        o.y = 0;
        const int k = (i <= a.n1 / 2) ? i : i - a.n1;
        const int ak = k < 0 ? -k : k;
        if (ak <= a.lmax)
            o = scale_c(X[fd.perm[k < 0 ? k + a.nd : k]], a.kf1[ak] * fm);
        return o;
    };
    if (!FULL) {
        for (int i = tid; i < a.n1; i += COL_THREADS)
            ec[i] = deconv(i);
        return;
    }
    constexpr int MAXV = col_maxv<T>();
    C y[MAXV];
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * COL_THREADS;
        if (i < a.n1)
            y[v] = deconv(i);
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * COL_THREADS;
        if (i < a.n1)
            X[i] = y[v];
    }
    __syncthreads();
    lds_fft<C, 1>(X, f1);
    for (int i = tid; i < a.n1; i += COL_THREADS)
        if (row_kept(i, a.n1, a.nrows, a.a_min))
            ec[i] = X[f1.perm[i]];
}

// FULL: E column (kept rows; the rest is zero) -> D column.  Otherwise E holds
// the theta spectrum already and only the deconvolution and nd transform run here.
template <typename T, bool FULL>
__global__ __launch_bounds__(COL_THREADS) void column_adj_kernel(
    const typename cx<T>::type *__restrict__ E, typename cx<T>::type *__restrict__ D, ColArgs a,
    ColFFT fd, ColFFT f1)
{
    using C = typename cx<T>::type;
    extern __shared__ unsigned char smem_raw[];
    C *X = reinterpret_cast<C *>(smem_raw);
    const int col = blockIdx.x, tid = threadIdx.x;
    const int m = col_m(a, col);
    const double fm = a.kf2[m < 0 ? -m : m];
    const C *ec = E + (size_t)col * a.n1;
    C *dc = D + (size_t)col * a.nd;
    if (FULL) {
        for (int i = tid; i < a.n1; i += COL_THREADS) {
            C v;
            v.x = 0;
            v.y = 0;
            if (row_kept(i, a.n1, a.nrows, a.a_min))
                v = ec[i];
            X[i] = v;
        }
        __syncthreads();
        lds_fft<C, -1>(X, f1);
    }
    // deconvolution: output i in [0, nd) <- theta frequency k
    auto deconv = [&](int i) {
        C o;
        o.x = 0;
        o.y = 0;
        const int k = (i <= a.nd / 2) ? i : i - a.nd;
        const int ak = k < 0 ? -k : k;
        if (ak <= a.lmax) {
            const int ka = k < 0 ? k + a.n1 : k;
            o = scale_c(FULL ? X[f1.perm[ka]] : ec[ka], a.kf1[ak] * fm);
        }
        return o;
    };
    if (FULL) {
        constexpr int MAXV = col_maxv<T>();
        C y[MAXV];
#pragma unroll
        for (int v = 0; v < MAXV; ++v) {
            const int i = tid + v * COL_THREADS;
            if (i < a.nd)
                y[v] = deconv(i);
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < MAXV; ++v) {
            const int i = tid + v * COL_THREADS;
            if (i < a.nd)
                X[i] = y[v];
        }
    } else {
        for (int i = tid; i < a.nd; i += COL_THREADS)
            X[i] = deconv(i);
    }
    __syncthreads();
    lds_fft<C, 1>(X, fd);
    for (int i = tid; i < a.nd; i += COL_THREADS)
        dc[i] = X[fd.perm[i]];
}

ColArgs col_args(const gsht_plan &p)
{
    ColArgs a;
    a.kf1 = p.kfac1;
    a.kf2 = p.kfac2;
    a.lmax = p.lmax;
    a.mmax = p.mmax;
    a.spin = p.spin;
    a.nd = p.nd;
    a.n1 = p.n1;
    a.nrows = p.nrows;
    a.a_min = p.a_min;
    return a;
}

template <typename T>
size_t col_lds(const gsht_plan &p)
{
    const int n = p.colmode == 2 ? std::max(p.nd, p.n1) : p.nd;
    return sizeof(typename cx<T>::type) * (size_t)n;
}

}  // namespace

hipError_t column_set_lds(const gsht_plan &p)
{
    hipError_t e = hipSuccess;
    if (p.prec == GSHT_F64) {
        const int b = (int)col_lds<double>(p);
        if (p.colmode == 2) {
            e = hipFuncSetAttribute((const void *)column_fwd_kernel<double, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, b);
            if (e == hipSuccess)
                e = hipFuncSetAttribute((const void *)column_adj_kernel<double, true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, b);
        } else {
            e = hipFuncSetAttribute((const void *)column_fwd_kernel<double, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, b);
            if (e == hipSuccess)
                e = hipFuncSetAttribute((const void *)column_adj_kernel<double, false>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, b);
        }
    } else {
        const int b = (int)col_lds<float>(p);
        if (p.colmode == 2) {
            e = hipFuncSetAttribute((const void *)column_fwd_kernel<float, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, b);
            if (e == hipSuccess)
                e = hipFuncSetAttribute((const void *)column_adj_kernel<float, true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, b);
        } else {
            e = hipFuncSetAttribute((const void *)column_fwd_kernel<float, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, b);
            if (e == hipSuccess)
                e = hipFuncSetAttribute((const void *)column_adj_kernel<float, false>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, b);
        }
    }
    return e;
}

hipError_t launch_column_fwd(const gsht_plan &p, hipStream_t s)
{
    const ColArgs a = col_args(p);
    const dim3 grd(p.ncol), blk(COL_THREADS);
    if (p.prec == GSHT_F64) {
        const size_t b = col_lds<double>(p);
        if (p.colmode == 2)
            hipLaunchKernelGGL((column_fwd_kernel<double, true>), grd, blk, b, s,
                               (const double2 *)p.D, (double2 *)p.E, a, p.cf_d, p.cf_1);
        else
            hipLaunchKernelGGL((column_fwd_kernel<double, false>), grd, blk, b, s,
                               (const double2 *)p.D, (double2 *)p.E, a, p.cf_d, p.cf_1);
    } else {
        const size_t b = col_lds<float>(p);
        if (p.colmode == 2)
            hipLaunchKernelGGL((column_fwd_kernel<float, true>), grd, blk, b, s,
                               (const float2 *)p.D, (float2 *)p.E, a, p.cf_d, p.cf_1);
        else
            hipLaunchKernelGGL((column_fwd_kernel<float, false>), grd, blk, b, s,
                               (const float2 *)p.D, (float2 *)p.E, a, p.cf_d, p.cf_1);
    }
    return hipGetLastError();
}

hipError_t launch_column_adj(const gsht_plan &p, hipStream_t s)
{
    const ColArgs a = col_args(p);
    const dim3 grd(p.ncol), blk(COL_THREADS);
    if (p.prec == GSHT_F64) {
        const size_t b = col_lds<double>(p);
        if (p.colmode == 2)
            hipLaunchKernelGGL((column_adj_kernel<double, true>), grd, blk, b, s,
                               (const double2 *)p.E, (double2 *)p.D, a, p.cf_d, p.cf_1);
        else
            hipLaunchKernelGGL((column_adj_kernel<double, false>), grd, blk, b, s,
                               (const double2 *)p.E, (double2 *)p.D, a, p.cf_d, p.cf_1);
    } else {
        const size_t b = col_lds<float>(p);
        if (p.colmode == 2)
            hipLaunchKernelGGL((column_adj_kernel<float, true>), grd, blk, b, s,
                               (const float2 *)p.E, (float2 *)p.D, a, p.cf_d, p.cf_1);
        else
            hipLaunchKernelGGL((column_adj_kernel<float, false>), grd, blk, b, s,
                               (const float2 *)p.E, (float2 *)p.D, a, p.cf_d, p.cf_1);
    }
    return hipGetLastError();
}

}  // namespace gsht

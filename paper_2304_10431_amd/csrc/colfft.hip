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
// 8, 4, 2, 3, 5, 7): pass i splits sub-transforms of length L into radix r_i
// butterflies of stride s = L / r_i, each followed by the twiddles w_L^(q j).  The
// result sits in digit-reversed order; a host-built table gives the LDS position of
// every frequency.  Twiddles come from per-pass tables in the working precision,
// read contiguously per butterfly.
#include <algorithm>

#include "gsht_internal.hpp"

namespace gsht {

namespace {

constexpr int COL_THREADS = 1024;

// largest radix of the in-LDS transforms (a radix-16 pass, 16 complex values plus 15
// twiddles, does not fit the 128 registers of either precision's workgroups)
constexpr int COL_MAXR = 8;

template <typename T> struct cx;
template <> struct cx<float> { using type = float2; };
template <> struct cx<double> { using type = double2; };
template <typename C> struct cx2;  // two complex values
template <> struct cx2<float2> { using type = float4; };
template <> struct cx2<double2> { using type = double4; };

// Mode 2 (split theta transform): threads per workgroup and the largest nd or
// n1 / 2 it takes; each thread stages up to col_half_maxn / threads values in
// registers.  FP32: two workgroups of 512 threads (2 x 66 KB of LDS at lmax 4096)
// share a CU.  FP64: one workgroup per CU (132 KB) of 1024 threads, so that four
// waves per SIMD hide the LDS latency of the passes (18 % faster than 512 threads
// with radix-16 passes).  Either way 16 waves per CU and 128 VGPRs.
template <typename T>
constexpr int col_half_threads()
{
    return sizeof(T) == 4 ? 512 : 1024;
}
template <typename T>
constexpr int col_half_waves()  // waves per SIMD
{
    return 4;
}
template <typename T>
constexpr int col_half_maxn()
{
    return sizeof(T) == 4 ? 17 * 512 : 20 * 512;
}

// FP64 mode-2 kernels are instantiated for every register slot count MAXV up to
// col_half_maxn / threads and launched with the smallest that holds the plan's
// transforms (the forward kernel's slots cover nh = n1 / 2, the adjoint's max(nd, nh)):
// slots sized for the largest case held 40 VGPRs per array and spilled 24 registers
// to scratch at lmax 4096, where 6 and 9 slots suffice (column forward 1.70 -> 1.61 ms,
// adjoint 1.72 -> 1.67 ms at sigma 1.5).  FP32 runs with the largest count: its 512
// threads leave it 128 registers for half the slots, and it does not spill.
template <typename T>
constexpr int col_half_maxv()
{
    return col_half_maxn<T>() / col_half_threads<T>();
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

// One decimation-in-frequency pass over NT threads: butterflies b < n / R over
// sub-transforms of length L = R s; butterfly (sub, j) reads positions
// sub L + j + t s, t < R, and its twiddles w_L^(q j) from tw[j (R - 1) + q - 1]
// (conjugated for DIR > 0): a lane's twiddles are contiguous.
template <typename C, int R, int DIR, int NT>
__device__ inline void dif_pass(C *X, const C *__restrict__ tw, int n, int s, int sh)
{
    const int L = R * s, nb = n / R;
    const double rs = 1.0 / (double)s;  // b / s by an FP64 product: exact for b < 2^26
    for (int b = threadIdx.x; b < nb; b += NT) {
        const int sub = (int)(((double)b + 0.5) * rs), j = b - sub * s;
        const int base = sub * L + j;
        C v[R];
#pragma unroll
        for (int t = 0; t < R; ++t)
            v[t] = X[lds_pos(base + t * s, sh)];
        dft<C, R, DIR>(v);
        if (j != 0) {
#pragma unroll
            for (int q = 1; q < R; ++q) {
                C w = tw[j * (R - 1) + q - 1];
                if (DIR > 0)
                    w.y = -w.y;
                const C a = v[q];
                v[q].x = a.x * w.x - a.y * w.y;
                v[q].y = a.x * w.y + a.y * w.x;
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t)
            X[lds_pos(base + t * s, sh)] = v[t];
    }
}

// Whole transform in LDS (the block must hold the column before the call; the
// result is in digit-reversed order when it returns, after a barrier).
template <typename C, int DIR, int NT>
__device__ void lds_fft(C *X, const ColFFT &f)
{
    int L = f.n;
    for (int p = 0; p < f.npass; ++p) {
        const int r = f.radix[p];
        const int s = L / r;
        const C *tw = reinterpret_cast<const C *>(f.tw) + f.twoff[p];
        switch (r) {
        case 8: dif_pass<C, 8, DIR, NT>(X, tw, f.n, s, f.psh); break;
        case 4: dif_pass<C, 4, DIR, NT>(X, tw, f.n, s, f.psh); break;
        case 2: dif_pass<C, 2, DIR, NT>(X, tw, f.n, s, f.psh); break;
        case 3: dif_pass<C, 3, DIR, NT>(X, tw, f.n, s, f.psh); break;
        case 5: dif_pass<C, 5, DIR, NT>(X, tw, f.n, s, f.psh); break;
        case 7: dif_pass<C, 7, DIR, NT>(X, tw, f.n, s, f.psh); break;
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

template <typename C>
__device__ inline C cmul(C a, C b)
{
    C o;
    o.x = a.x * b.x - a.y * b.y;
    o.y = a.x * b.y + a.y * b.x;
    return o;
}

template <typename C>
__device__ inline C cmulc(C a, C b)  // a * conj(b)
{
    C o;
    o.x = a.x * b.x + a.y * b.y;
    o.y = a.y * b.x - a.x * b.y;
    return o;
}

// LDS of mode 2: the column buffer (the transforms of lengths nd and nh = n1 / 2).
__host__ __device__ inline int col_half_lds_n(int nd, int nh) { return nd > nh ? nd : nh; }

struct ColArgs {
    const double *kf1, *kf2;
    int lmax, mmax, spin, nd, n1, nrows, a_min;
};

__device__ inline int col_m(const ColArgs &a, int col) { return a.spin ? col - a.mmax : col; }

// Rows 2i (value ev) and 2i + 1 (od) of an E column, those of them the grid keeps;
// one 2-element store when both are kept (E columns have even length, so the pair is
// aligned to its own size).
template <typename C>
__device__ inline void store_rows(C *ec, int i, C ev, C od, const ColArgs &a)
{
    using C2 = typename cx2<C>::type;
    const bool ke = row_kept(2 * i, a.n1, a.nrows, a.a_min);
    const bool ko = row_kept(2 * i + 1, a.n1, a.nrows, a.a_min);
    if (ke && ko) {
        C2 p;
        p.x = ev.x;
        p.y = ev.y;
        p.z = od.x;
        p.w = od.y;
        reinterpret_cast<C2 *>(ec)[i] = p;
    } else if (ke) {
        ec[2 * i] = ev;
    } else if (ko) {
        ec[2 * i + 1] = od;
    }
}

// Rows 2i and 2i + 1 of an E column as (ev, od), zero where the grid keeps no row.
template <typename C>
__device__ inline void load_rows(const C *ec, int i, C &ev, C &od, const ColArgs &a)
{
    using C2 = typename cx2<C>::type;
    const bool ke = row_kept(2 * i, a.n1, a.nrows, a.a_min);
    const bool ko = row_kept(2 * i + 1, a.n1, a.nrows, a.a_min);
    ev.x = ev.y = od.x = od.y = 0;
    if (ke && ko) {
        const C2 p = reinterpret_cast<const C2 *>(ec)[i];
        ev.x = p.x;
        ev.y = p.y;
        od.x = p.z;
        od.y = p.w;
    } else if (ke) {
        ev = ec[2 * i];
    } else if (ko) {
        od = ec[2 * i + 1];
    }
}

// Mode 2, D column -> E column (kept rows).  The oversampled theta transform is
// split by output parity: with nh = n1 / 2 and the spectrum c_k, |k| <= lmax,
//   E[2a'] = sum_k c_k e^{2 pi i k a' / nh},  E[2a' + 1] = sum_k (c_k t^k) e^{2 pi i k a' / nh},
// t = e^{2 pi i / n1}: two length-nh transforms of the spectra folded modulo nh (at
// most two k per residue, since nh > lmax), so the LDS buffer holds max(nd, nh)
// values.  twist[k] = e^{-2 pi i k / n1}, k < n1.
template <typename T, int NT, int MAXV>
__global__ __launch_bounds__(NT, col_half_waves<T>()) void column_fwd_half_kernel(
    const typename cx<T>::type *__restrict__ D, typename cx<T>::type *__restrict__ E, ColArgs a,
    ColFFT fd, ColFFT fh, const typename cx<T>::type *__restrict__ twist)
{
    using C = typename cx<T>::type;
    extern __shared__ unsigned char smem_raw[];
    C *X = reinterpret_cast<C *>(smem_raw);
    const int sh = fd.psh;  // LDS padding shift
    const int col = blockIdx.x, tid = threadIdx.x, nh = fh.n;
    const int m = col_m(a, col);
    const double fm = a.kf2[m < 0 ? -m : m];
    const C *dc = D + (size_t)col * a.nd;
    C *ec = E + (size_t)col * a.n1;
    for (int i = tid; i < a.nd; i += NT)
        X[lds_pos(i, sh)] = dc[i];
    __syncthreads();
    lds_fft<C, -1, NT>(X, fd);
    auto chat = [&](int k) {
        const int ak = k < 0 ? -k : k;
        return scale_c(X[lds_pos(fd.perm[k < 0 ? k + a.nd : k], sh)], a.kf1[ak] * fm);
    };
    // Fold: residue i < nh receives c_i (i <= lmax) and c_{i - nh} (i >= nh - lmax);
    // absent terms count as zero.  The even-row input is ye = c_i + c_{i-nh}, the
    // odd-row input t^i (c_i - c_{i-nh}) (t^{-nh} = -1).  Both are formed in
    // registers before the odd input overwrites the spectrum in LDS; ye stays there
    // until the even transform.
    const int ov0 = nh - a.lmax;
    C ye[MAXV], yd[MAXV];
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * NT;
        ye[v].x = ye[v].y = 0;
        yd[v] = ye[v];
        if (i < nh) {
            C c1, c2;
            c1.x = c1.y = 0;
            c2 = c1;
            if (i <= a.lmax)
                c1 = chat(i);
            if (i >= ov0)
                c2 = chat(i - nh);
            ye[v] = cadd(c1, c2);
            yd[v] = csub(c1, c2);
        }
    }
    __syncthreads();
    // odd rows
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * NT;
        if (i < nh)
            X[lds_pos(i, sh)] = cmulc(yd[v], twist[i]);
    }
    __syncthreads();
    lds_fft<C, 1, NT>(X, fh);
    // the odd rows wait in registers (in place of ye) until the even rows are done,
    // so that rows 2i and 2i + 1 leave as one contiguous store
    C od[MAXV];
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * NT;
        od[v].x = od[v].y = 0;
        if (i < nh)
            od[v] = X[lds_pos(fh.perm[i], sh)];
    }
    __syncthreads();
    // even rows
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * NT;
        if (i < nh)
            X[lds_pos(i, sh)] = ye[v];
    }
    __syncthreads();
    lds_fft<C, 1, NT>(X, fh);
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * NT;
        if (i < nh)
            store_rows(ec, i, X[lds_pos(fh.perm[i], sh)], od[v], a);
    }
}

// Mode 2, E column (kept rows; the rest counts as zero) -> D column: the transpose
// of column_fwd_half_kernel (odd rows first, then even rows).
template <typename T, int NT, int MAXV>
__global__ __launch_bounds__(NT, col_half_waves<T>()) void column_adj_half_kernel(
    const typename cx<T>::type *__restrict__ E, typename cx<T>::type *__restrict__ D, ColArgs a,
    ColFFT fd, ColFFT fh, const typename cx<T>::type *__restrict__ twist)
{
    using C = typename cx<T>::type;
    extern __shared__ unsigned char smem_raw[];
    C *X = reinterpret_cast<C *>(smem_raw);
    const int sh = fd.psh;  // LDS padding shift
    const int col = blockIdx.x, tid = threadIdx.x, nh = fh.n;
    const int m = col_m(a, col);
    const double fm = a.kf2[m < 0 ? -m : m];
    const C *ec = E + (size_t)col * a.n1;
    C *dc = D + (size_t)col * a.nd;
    // theta frequency k of output i (|k| <= lmax contributes) and its residue mod nh
    auto freq = [&](int i, int &k, int &kh) {
        k = (i <= a.nd / 2) ? i : i - a.nd;
        kh = k % nh;
        if (kh < 0)
            kh += nh;
        return (k < 0 ? -k : k) <= a.lmax;
    };
    // rows 2i and 2i + 1 arrive as one load; the odd rows go first, the even rows
    // wait in registers
    C ev[MAXV];
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * NT;
        ev[v].x = ev[v].y = 0;
        if (i < nh) {
            C od;
            load_rows(ec, i, ev[v], od, a);
            X[lds_pos(i, sh)] = od;
        }
    }
    __syncthreads();
    lds_fft<C, -1, NT>(X, fh);
    C acc[MAXV];
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * NT;
        acc[v].x = acc[v].y = 0;
        int k, kh;
        if (i < a.nd && freq(i, k, kh))
            acc[v] = cmul(X[lds_pos(fh.perm[kh], sh)], twist[k < 0 ? k + a.n1 : k]);
    }
    __syncthreads();
    // even rows
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * NT;
        if (i < nh)
            X[lds_pos(i, sh)] = ev[v];
    }
    __syncthreads();
    lds_fft<C, -1, NT>(X, fh);
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * NT;
        int k, kh;
        if (i < a.nd && freq(i, k, kh))
            acc[v] = scale_c(cadd(acc[v], X[lds_pos(fh.perm[kh], sh)]), a.kf1[k < 0 ? -k : k] * fm);
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        const int i = tid + v * NT;
        if (i < a.nd)
            X[lds_pos(i, sh)] = acc[v];
    }
    __syncthreads();
    lds_fft<C, 1, NT>(X, fd);
    for (int i = tid; i < a.nd; i += NT)
        dc[i] = X[lds_pos(fd.perm[i], sh)];
}

// Mode 1, D column -> zero-padded, deconvolved spectrum over all n1 entries (the
// theta transform follows in the library FFT).
template <typename T>
__global__ __launch_bounds__(COL_THREADS) void column_fwd_kernel(
    const typename cx<T>::type *__restrict__ D, typename cx<T>::type *__restrict__ E, ColArgs a,
    ColFFT fd)
{
    using C = typename cx<T>::type;
    extern __shared__ unsigned char smem_raw[];
    C *X = reinterpret_cast<C *>(smem_raw);
    const int sh = fd.psh;  // LDS padding shift
    const int col = blockIdx.x, tid = threadIdx.x;
    const int m = col_m(a, col);
    const double fm = a.kf2[m < 0 ? -m : m];
    const C *dc = D + (size_t)col * a.nd;
    C *ec = E + (size_t)col * a.n1;
    for (int i = tid; i < a.nd; i += COL_THREADS)
        X[lds_pos(i, sh)] = dc[i];
    __syncthreads();
    lds_fft<C, -1, COL_THREADS>(X, fd);
    for (int i = tid; i < a.n1; i += COL_THREADS) {
        C o;
        o.x = 0;
        o.y = 0;
        const int k = (i <= a.n1 / 2) ? i : i - a.n1;
        const int ak = k < 0 ? -k : k;
        if (ak <= a.lmax)
            o = scale_c(X[lds_pos(fd.perm[k < 0 ? k + a.nd : k], sh)], a.kf1[ak] * fm);
        ec[i] = o;
    }
}

// Mode 1, theta spectrum E^ -> deconvolution and nd transform -> D column.
template <typename T>
__global__ __launch_bounds__(COL_THREADS) void column_adj_kernel(
    const typename cx<T>::type *__restrict__ E, typename cx<T>::type *__restrict__ D, ColArgs a,
    ColFFT fd)
{
    using C = typename cx<T>::type;
    extern __shared__ unsigned char smem_raw[];
    C *X = reinterpret_cast<C *>(smem_raw);
    const int sh = fd.psh;  // LDS padding shift
    const int col = blockIdx.x, tid = threadIdx.x;
    const int m = col_m(a, col);
    const double fm = a.kf2[m < 0 ? -m : m];
    const C *ec = E + (size_t)col * a.n1;
    C *dc = D + (size_t)col * a.nd;
    for (int i = tid; i < a.nd; i += COL_THREADS) {
        C o;
        o.x = 0;
        o.y = 0;
        const int k = (i <= a.nd / 2) ? i : i - a.nd;
        const int ak = k < 0 ? -k : k;
        if (ak <= a.lmax)
            o = scale_c(ec[k < 0 ? k + a.n1 : k], a.kf1[ak] * fm);
        X[lds_pos(i, sh)] = o;
    }
    __syncthreads();
    lds_fft<C, 1, COL_THREADS>(X, fd);
    for (int i = tid; i < a.nd; i += COL_THREADS)
        dc[i] = X[lds_pos(fd.perm[i], sh)];
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
    const int sh = p.lds_psh;
    const int n = p.colmode == 2 ? lds_pad_n(col_half_lds_n(p.nd, p.n1 / 2), sh)
                                 : lds_pad_n(p.nd, sh);
    return sizeof(typename cx<T>::type) * (size_t)n;
}

// Register slots of the mode-2 kernels for this plan (see col_half_maxv).
template <typename T>
int half_slots(const gsht_plan &p, bool adjoint)
{
    constexpr int NT = col_half_threads<T>();
    const int nh = p.n1 / 2, n = adjoint ? (p.nd > nh ? p.nd : nh) : nh;
    const int v = (n + NT - 1) / NT;
    return v < 1 ? 1 : v;
}

// Calls f with the kernel instance of MV = v slots (MV counts down from the largest;
// FP32 has only the largest).
template <typename T, int MV, typename F>
hipError_t with_fwd_half(int v, F &&f)
{
    if constexpr (sizeof(T) == 8 && MV > 1)
        if (v < MV)
            return with_fwd_half<T, MV - 1>(v, f);
    return f(column_fwd_half_kernel<T, col_half_threads<T>(), MV>);
}
template <typename T, int MV, typename F>
hipError_t with_adj_half(int v, F &&f)
{
    if constexpr (sizeof(T) == 8 && MV > 1)
        if (v < MV)
            return with_adj_half<T, MV - 1>(v, f);
    return f(column_adj_half_kernel<T, col_half_threads<T>(), MV>);
}

template <typename T>
hipError_t set_lds(const gsht_plan &p)
{
    const int b = (int)col_lds<T>(p);
    hipError_t e;
    if (p.colmode == 2) {
        auto attr = [&](auto kern) {
            return hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, b);
        };
        e = with_fwd_half<T, col_half_maxv<T>()>(half_slots<T>(p, false), attr);
        if (e == hipSuccess)
            e = with_adj_half<T, col_half_maxv<T>()>(half_slots<T>(p, true), attr);
    } else {
        e = hipFuncSetAttribute((const void *)column_fwd_kernel<T>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, b);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)column_adj_kernel<T>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, b);
    }
    return e;
}

template <typename T>
void launch_fwd(const gsht_plan &p, hipStream_t s)
{
    using C = typename cx<T>::type;
    const ColArgs a = col_args(p);
    const size_t b = col_lds<T>(p);
    if (p.colmode == 2) {
        constexpr int NT = col_half_threads<T>();
        (void)with_fwd_half<T, col_half_maxv<T>()>(half_slots<T>(p, false), [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(p.ncol), dim3(NT), b, s, (const C *)p.D, (C *)p.E, a,
                               p.cf_d, p.cf_h, (const C *)p.twist);
            return hipSuccess;
        });
    } else {
        hipLaunchKernelGGL((column_fwd_kernel<T>), dim3(p.ncol), dim3(COL_THREADS), b, s,
                           (const C *)p.D, (C *)p.E, a, p.cf_d);
    }
}

template <typename T>
void launch_adj(const gsht_plan &p, hipStream_t s)
{
    using C = typename cx<T>::type;
    const ColArgs a = col_args(p);
    const size_t b = col_lds<T>(p);
    if (p.colmode == 2) {
        constexpr int NT = col_half_threads<T>();
        (void)with_adj_half<T, col_half_maxv<T>()>(half_slots<T>(p, true), [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(p.ncol), dim3(NT), b, s, (const C *)p.E, (C *)p.D, a,
                               p.cf_d, p.cf_h, (const C *)p.twist);
            return hipSuccess;
        });
    } else {
        hipLaunchKernelGGL((column_adj_kernel<T>), dim3(p.ncol), dim3(COL_THREADS), b, s,
                           (const C *)p.E, (C *)p.D, a, p.cf_d);
    }
}

}  // namespace

hipError_t column_set_lds(const gsht_plan &p)
{
    return p.prec == GSHT_F64 ? set_lds<double>(p) : set_lds<float>(p);
}

int column_half_maxn(int prec) { return prec == GSHT_F64 ? col_half_maxn<double>() : col_half_maxn<float>(); }

int column_max_radix(int) { return COL_MAXR; }

size_t column_lds_bytes(const gsht_plan &p)
{
    return p.prec == GSHT_F64 ? col_lds<double>(p) : col_lds<float>(p);
}

hipError_t launch_column_fwd(const gsht_plan &p, hipStream_t s)
{
    if (p.prec == GSHT_F64)
        launch_fwd<double>(p, s);
    else
        launch_fwd<float>(p, s);
    return hipGetLastError();
}

hipError_t launch_column_adj(const gsht_plan &p, hipStream_t s)
{
    if (p.prec == GSHT_F64)
        launch_adj<double>(p, s);
    else
        launch_adj<float>(p, s);
    return hipGetLastError();
}

}  // namespace gsht

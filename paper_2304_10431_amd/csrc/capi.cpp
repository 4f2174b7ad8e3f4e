// C ABI of the gfx950 general-SHT library: argument validation, plan
// construction (grid sizes, kernel parameters, deconvolution tables, bin sort,
// rocFFT plans, workspace) and the order of the steps of Sect. 3.
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gsht_internal.hpp"

namespace gsht {
std::vector<StartInfo> make_start_info(int lmax, int mmax, int spin);
}

using namespace gsht;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int ok()
{
    g_last_error.clear();
    return GSHT_OK;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(GSHT_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));             \
    } while (0)

#define FFT_TRY(expr)                                                                          \
    do {                                                                                       \
        rocfft_status s_ = (expr);                                                             \
        if (s_ != rocfft_status_success)                                                       \
            return fail(GSHT_EHIP, "%s failed: rocfft status %d", #expr, (int)s_);             \
    } while (0)

std::once_flag g_fft_once;

// ---- device scratch of the allocation-free entry point ------------------------
// One fixed array per device, in the code object's global memory: the Legendre
// tables, the start data and the adjoint's accumulators of one
// gsht_legendre_rings_adjoint_noalloc call live here instead of in allocations.  Host
// code must not pass the array's name to a kernel (it is a host-side stand-in, not a
// device address): its address on each device comes from hipGetSymbolAddress, taken
// once per device with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
// host copies of the start data most recently sent to each device's scratch (kept
// until the next call on that device)
std::vector<StartInfo> g_scratch_start[kMaxDevices];

int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(GSHT_EUNSUPPORTED, "device %d is beyond the %d devices the scratch table covers",
                    dev, kMaxDevices);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(GSHT_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return GSHT_OK;
}

bool smooth7(long n)
{
    if (n < 1)
        return false;
    for (long f : {2L, 3L, 5L, 7L})
        while (n % f == 0)
            n /= f;
    return n == 1;
}

long next_smooth_even(long n)
{
    if (n < 2)
        n = 2;
    while (!(smooth7(n) && n % 2 == 0))
        ++n;
    return n;
}

// Oversampled torus length: the smallest 2^k, 3 * 2^k or 5 * 2^k (k >= 1) that is
// at least 0.999 * target (an oversampling factor of 2 may thus become 1.998, which
// changes the kernel error negligibly) and at least floor_n.  These lengths run as
// one or two passes in rocFFT, unlike lengths with several factors of 7.
long fft_size(double target, long floor_n)
{
    long best = 0;
    for (long f : {2L, 3L, 5L}) {
        long n = f;
        while (n < 0.999 * target || n < floor_n || n % 2)
            n *= 2;
        if (best == 0 || n < best)
            best = n;
    }
    return best;
}

// Kernel settings by oversampling factor sigma (Sect. 3: sigma between about 1.2
// and 2 trades grid size against kernel support).  err[w] is the relative L2 error
// of the 2-D type-2 NUFFT with support w and beta = beta_per_w * w, measured for
// w = 4..16 on random Fourier series (81 x 81 modes, 2000 random points, torus of
// sigma * 81 cells); beta_per_w is the value that minimised the error for mid-range w
// (for sigma = 2 it matches the 2.3 w of the exponential-of-semicircle literature).
// The sigma = 2 row lists, at w = 4, 5 and 13..16, the error at the best beta near
// 2.3 w; at 2.3 w itself it is up to 1.6 times larger there (w = 16: 1.9e-14, the
// test's own floor), which the factor 2 margin of choose_w absorbs for every
// epsilon a plan accepts.  tests/test_es_table.py recomputes every entry with the
// plain FP64 CPU NUFFT on the same draw.
struct EsSetting {
    double sigma, beta_per_w;
    double err[17];
};
const EsSetting kEs[3] = {
    {2.0, 2.3, {0, 0, 0, 0, 7.8e-4, 8.8e-5, 9.7e-6, 1.2e-6, 1.5e-7, 1.7e-8, 2.0e-9, 2.0e-10,
                2.0e-11, 2.1e-12, 2.0e-13, 2.4e-14, 3.0e-15}},
    {1.5, 2.05, {0, 0, 0, 0, 3.9e-3, 5.6e-4, 7.6e-5, 1.1e-5, 2.0e-6, 3.9e-7, 7.2e-8, 1.2e-8,
                 1.8e-9, 2.5e-10, 3.8e-11, 7.4e-12, 1.5e-12}},
    {1.25, 1.85, {0, 0, 0, 0, 1.3e-2, 2.9e-3, 5.9e-4, 1.1e-4, 2.5e-5, 7.5e-6, 2.3e-6, 6.4e-7,
                  1.6e-7, 3.3e-8, 6.2e-9, 1.2e-9, 4.0e-10}},
};
constexpr int kNumEs = 3;

// Interior-tap kernel weights of FP64 plans as polynomials.  Tap i of a point at
// cell offset dx in (w/2 - 1, w/2] weighs psi((dx - i) 2 / w); with y = 2 dx - w + 1
// in (-1, 1] that is a smooth function of y for 0 < i < w - 1 (the kernel's
// square-root edges lie outside those intervals; the two edge taps keep the exact
// formula).  Chebyshev interpolation at pdeg + 1 nodes in long double, converted to
// monomial coefficients; accepted only if the double Horner evaluation stays within
// 5e-15 of the kernel at 2001 points per tap (else the plan uses the exact formula).
bool es_poly_fit(int w, double beta, std::vector<double> &coef)
{
    const int D = es_pdeg_rt(w), N = D + 1;
    coef.assign((size_t)w * N, 0.0);
    const long double pi = 3.14159265358979323846264338327950288L;
    auto psi = [&](long double z) {
        long double t = 1.0L - z * z;
        if (t < 0)
            t = 0;
        return expl((long double)beta * (sqrtl(t) - 1.0L));
    };
    auto zof = [&](long double y, int i) {
        const long double dx = (y + 1.0L) / 2.0L + 0.5L * w - 1.0L;
        return (dx - i) * 2.0L / w;
    };
    // monomial coefficients of the Chebyshev polynomials T_0 .. T_D
    std::vector<long double> tm((size_t)N * N, 0.0L), f(N), c(N);
    tm[0] = 1.0L;
    if (N > 1)
        tm[(size_t)N + 1] = 1.0L;
    for (int k = 2; k < N; ++k)
        for (int m = 0; m < N; ++m)
            tm[(size_t)k * N + m] = (m > 0 ? 2.0L * tm[(size_t)(k - 1) * N + m - 1] : 0.0L) -
                                    tm[(size_t)(k - 2) * N + m];
    for (int i = 1; i < w - 1; ++i) {
        for (int j = 0; j < N; ++j)
            f[j] = psi(zof(cosl(pi * (j + 0.5L) / N), i));
        for (int k = 0; k < N; ++k) {
            long double acc = 0.0L;
            for (int j = 0; j < N; ++j)
                acc += f[j] * cosl(pi * k * (j + 0.5L) / N);
            c[k] = 2.0L * acc / N;
        }
        c[0] *= 0.5L;
        for (int m = 0; m < N; ++m) {
            long double a = 0.0L;
            for (int k = m; k < N; ++k)
                a += c[k] * tm[(size_t)k * N + m];
            coef[(size_t)i * N + m] = (double)a;
        }
        for (int t = 0; t <= 2000; ++t) {
            const double y = -1.0 + t / 1000.0;
            double v = coef[(size_t)i * N + D];
            for (int k = D - 1; k >= 0; --k)
                v = std::fma(v, y, coef[(size_t)i * N + k]);
            if (fabsl((long double)v - psi(zof(y, i))) > 5e-15L)
                return false;
        }
    }
    return true;
}

// Smallest support whose calibrated error is at most eps / 2 (a transform's own
// relative error then measures about the table's value: at sigma 1.5, w = 14 and
// eps = 1e-10 the benchmark's sampled errors are 6e-12 for the synthesis and 3e-11
// for the adjoint).  If none up to wmax is: wmax for the default sigma = 2 (the
// closest the plan gets), 0 (not reachable) for the others.
int choose_w(double eps, int wmax, int set)
{
    for (int w = 4; w <= wmax; ++w)
        if (kEs[set].err[w] <= 0.5 * eps)
            return w;
    return set == 0 ? wmax : 0;
}

int es_set_of(double sigma)
{
    for (int i = 0; i < kNumEs; ++i)
        if (std::fabs(sigma - kEs[i].sigma) < 1e-9)
            return i;
    return -1;
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &wt)
{
    x.assign(n, 0.0);
    wt.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double pp = 0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            pp = n * (z * p0 - p1) / (z * z - 1.0);
            const double dz = p0 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16)
                break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        wt[i] = wt[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

// h / psihat(k) for k = 0..kmax on an n-point periodic grid:
//   psihat(k) = (w h / 2) J(k),  J(k) = int_{-1}^{1} exp(beta (sqrt(1 - z^2) - 1)) cos(pi k w z / n) dz
// so h / psihat(k) = 2 / (w J(k)).
std::vector<double> deconv_table(int kmax, int n, int w, double beta, double extra)
{
    const int nq = std::max(96, 4 * w + 64);
    std::vector<double> z, wt;
    gauss_legendre(nq, z, wt);
    std::vector<double> phi(nq);
    for (int i = 0; i < nq; ++i)
        phi[i] = wt[i] * exp(beta * (sqrt(std::max(0.0, 1.0 - z[i] * z[i])) - 1.0));
    std::vector<double> out((size_t)kmax + 1);
    for (int k = 0; k <= kmax; ++k) {
        double J = 0;
        const double f = M_PI * (double)k * (double)w / (double)n;
        for (int i = 0; i < nq; ++i)
            J += phi[i] * cos(f * z[i]);
        out[(size_t)k] = extra * 2.0 / ((double)w * J);
    }
    return out;
}

int check_common(int lmax, int mmax, int spin, int64_t npts, double eps, int prec)
{
    if (prec != GSHT_F64 && prec != GSHT_F32)
        return fail(GSHT_EINVAL, "precision must be GSHT_F64 (0) or GSHT_F32 (1), got %d", prec);
    if (lmax < 0 || lmax > 32766)
        return fail(GSHT_EINVAL, "lmax must be in [0, 32766], got %d", lmax);
    if (mmax < 0 || mmax > lmax)
        return fail(GSHT_EINVAL, "mmax must be in [0, lmax], got mmax=%d lmax=%d", mmax, lmax);
    if (spin < 0 || spin > lmax)
        return fail(GSHT_EINVAL, "spin must be in [0, lmax], got spin=%d lmax=%d", spin, lmax);
    if (npts < 0)
        return fail(GSHT_EINVAL, "npts must be >= 0, got %lld", (long long)npts);
    if (npts >= (int64_t)1 << 31)
        return fail(GSHT_EUNSUPPORTED, "npts must be < 2^31, got %lld", (long long)npts);
    const double lo = prec == GSHT_F64 ? 1e-13 : 1e-5;
    if (!(eps >= lo && eps <= 0.1))
        return fail(GSHT_EINVAL, "epsilon must be in [%g, 0.1] for this precision, got %g", lo, eps);
    return GSHT_OK;
}

int64_t workspace_cap()
{
    const char *e = getenv("GSHT_MAX_WORKSPACE_BYTES");
    if (!e || !*e)
        return INT64_MAX;
    return (int64_t)strtoll(e, nullptr, 10);
}

template <typename T>
int dev_alloc(gsht_plan *p, T **ptr, size_t bytes)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(GSHT_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    p->allocations.push_back(q);
    *ptr = (T *)q;
    return GSHT_OK;
}

void free_plan(gsht_plan *p)
{
    if (!p)
        return;
    (void)hipDeviceSynchronize();
    for (FFTPlan *f : {&p->fD_fwd, &p->fD_inv, &p->fT_inv, &p->fT_fwd, &p->fP_inv, &p->fP_fwd}) {
        if (f->info)
            rocfft_execution_info_destroy(f->info);
        if (f->plan)
            rocfft_plan_destroy(f->plan);
    }
    for (void *q : p->allocations)
        (void)hipFree(q);
    for (int i = 0; i < 2 * ST_COUNT; ++i)
        if (p->ev[i])
            (void)hipEventDestroy(p->ev[i]);
    delete p;
}

int make_fft(FFTPlan &f, rocfft_transform_type type, rocfft_result_placement place, int prec,
             size_t len, size_t batch)
{
    const rocfft_precision rp = prec == GSHT_F64 ? rocfft_precision_double : rocfft_precision_single;
    FFT_TRY(rocfft_plan_create(&f.plan, place, type, rp, 1, &len, batch, nullptr));
    FFT_TRY(rocfft_plan_get_work_buffer_size(f.plan, &f.work_bytes));
    FFT_TRY(rocfft_execution_info_create(&f.info));
    return GSHT_OK;
}

int run_fft(const FFTPlan &f, void *in, void *out, void *work, size_t work_bytes, hipStream_t s)
{
    FFT_TRY(rocfft_execution_info_set_stream(f.info, s));
    if (f.work_bytes)
        FFT_TRY(rocfft_execution_info_set_work_buffer(f.info, work, work_bytes));
    void *ib[1] = {in};
    void *ob[1] = {out};
    FFT_TRY(rocfft_execute(f.plan, ib, out ? ob : nullptr, f.info));
    return GSHT_OK;
}

// Compute grid sizes and kernel parameters (host only).
void choose_sizes(gsht_plan *p)
{
    p->ncomp = p->spin ? 2 : 1;
    p->nalm = (int64_t)(p->mmax + 1) * (p->lmax + 1) - (int64_t)p->mmax * (p->mmax + 1) / 2;
    long nt = std::max(p->lmax + 2, 2);
    while (!smooth7(2 * nt - 2))
        ++nt;
    p->ntheta = (int)nt;
    p->nd = 2 * p->ntheta - 2;
    p->w = choose_w(p->eps, p->prec == GSHT_F64 ? 16 : 8, p->es_set);
    if (p->w == 0)
        return;  // not reachable at this sigma; the caller reports it
    p->beta = kEs[p->es_set].beta_per_w * p->w;
    const double sigma = kEs[p->es_set].sigma;
    p->n1 = (int)fft_size(sigma * (2 * p->lmax + 1), std::max(2 * p->w + 4, 2 * p->lmax + 2));
    p->n2 = (int)fft_size(sigma * (2 * p->mmax + 1), std::max(2 * p->w + 4, 2 * p->mmax + 2));
    p->a_min = -(p->w / 2);
    p->nrows = p->n1 / 2 + p->w + 2;
    p->t1 = 32;
    p->t2 = 32;
    if (p->tile_req > 0)  // tile edge chosen by the caller (tuned plans) or GSHT_TILE
        p->t1 = p->t2 = p->tile_req;
    else if (const char *e = getenv("GSHT_TILE"))
        p->t1 = p->t2 = atoi(e);
    p->nt1 = (p->nrows + p->t1 - 1) / p->t1;
    p->nt2 = (p->n2 + p->t2 - 1) / p->t2;
    p->ntiles = (int64_t)p->nt1 * p->nt2;
    // order the points of a tile by their first kernel cell when the keys fit int32
    // (GSHT_CELL_SORT=0 keeps tile order for testing)
    p->cell_sort = p->ntiles * p->t1 * p->t2 < ((int64_t)1 << 31);
    if (const char *e = getenv("GSHT_CELL_SORT"))
        p->cell_sort = p->cell_sort && atoi(e) != 0;
    p->ncol = p->spin ? 2 * p->mmax + 1 : p->mmax + 1;
    p->npairs = (p->ntheta + 1) / 2;
}

// Allocate the Legendre tables and upload the start data and deconvolution tables.
int setup_legendre(gsht_plan *p, hipStream_t s, bool with_deconv)
{
    int rc;
    if ((rc = dev_alloc(p, &p->leg.ab, sizeof(double2) * (size_t)p->nalm)) != GSHT_OK) return rc;
    if ((rc = dev_alloc(p, &p->leg.norm, sizeof(double) * (size_t)p->nalm)) != GSHT_OK) return rc;
    if ((rc = dev_alloc(p, &p->leg.start, sizeof(StartInfo) * (size_t)(p->mmax + 1))) != GSHT_OK)
        return rc;
    if ((rc = dev_alloc(p, &p->uprep, sizeof(double) * 2 * p->ncomp * (size_t)p->nalm)) != GSHT_OK)
        return rc;
    if ((rc = dev_alloc(p, &p->acc, sizeof(double) * 2 * p->ncomp * (size_t)p->nalm)) != GSHT_OK)
        return rc;
    // Launch shapes of the Legendre kernels; GSHT_SYN_R, GSHT_ADJ_R and GSHT_ADJ_B
    // override the defaults for tuning (synthesis R in {1, 2, 4}; adjoint (R, B) in
    // {(1,8), (2,8), (2,4), (4,4), (3,8), (3,4), (4,8)}).
    {
        const char *sr = getenv("GSHT_SYN_R"), *ar = getenv("GSHT_ADJ_R"), *ab = getenv("GSHT_ADJ_B");
        const int r1 = sr ? atoi(sr) : p->syn_r;
        const int r2 = ar ? atoi(ar) : p->adj_r, b = ab ? atoi(ab) : p->adj_b;
        const int key = 100 * r2 + b;
        if ((r1 != 1 && r1 != 2 && r1 != 4) ||
            (key != 108 && key != 208 && key != 204 && key != 404 && key != 308 && key != 408 &&
             key != 304))
            return fail(GSHT_EINVAL, "unsupported Legendre launch shape syn_r=%d adj_r=%d adj_b=%d",
                        r1, r2, b);
        p->syn_r = r1;
        p->adj_r = r2;
        p->adj_b = b;
    }
    p->syn_nchunk = (p->npairs + 64 * p->syn_r - 1) / (64 * p->syn_r);
    p->adj_nchunk = (p->npairs + 64 * p->adj_r - 1) / (64 * p->adj_r);
    if ((rc = dev_alloc(p, &p->leg.lfirst_syn,
                        sizeof(int32_t) * (size_t)(p->mmax + 1) * p->syn_nchunk)) != GSHT_OK)
        return rc;
    if ((rc = dev_alloc(p, &p->leg.lfirst_adj,
                        sizeof(int32_t) * (size_t)(p->mmax + 1) * p->adj_nchunk)) != GSHT_OK)
        return rc;
    std::vector<StartInfo> si = make_start_info(p->lmax, p->mmax, p->spin);
    HIP_TRY(hipMemcpyAsync(p->leg.start, si.data(), sizeof(StartInfo) * si.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(launch_leg_tables(*p, s));
    HIP_TRY(launch_leg_live(*p, s));
    if (with_deconv) {
        std::vector<double> k1 = deconv_table(p->lmax, p->n1, p->w, p->beta, 1.0 / p->nd);
        std::vector<double> k2 = deconv_table(p->mmax, p->n2, p->w, p->beta, 1.0);
        if ((rc = dev_alloc(p, &p->kfac1, sizeof(double) * k1.size())) != GSHT_OK) return rc;
        if ((rc = dev_alloc(p, &p->kfac2, sizeof(double) * k2.size())) != GSHT_OK) return rc;
        HIP_TRY(hipMemcpyAsync(p->kfac1, k1.data(), sizeof(double) * k1.size(),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(p->kfac2, k2.data(), sizeof(double) * k2.size(),
                               hipMemcpyHostToDevice, s));
    }
    // the host vectors above are synchronised before they go out of scope
    HIP_TRY(hipStreamSynchronize(s));
    return GSHT_OK;
}

size_t csize(int prec) { return prec == GSHT_F64 ? 16 : 8; }

int col_maxr(const gsht_plan *p) { return column_max_radix(p->prec); }

// Radices of an in-LDS transform of length n (largest first, none above maxr, the
// largest radix the kernels are built with), or false if n has a prime factor above
// 7 or needs more than COL_MAXP passes.
bool col_radices(int n, std::vector<int> &rad, int maxr)
{
    rad.clear();
    int m = n;
    for (int f : {7, 5, 3})
        while (m % f == 0) {
            rad.push_back(f);
            m /= f;
        }
    while (m % maxr == 0) {
        rad.push_back(maxr);
        m /= maxr;
    }
    for (int f : {8, 4, 2})
        if (f < maxr && m % f == 0) {
            rad.push_back(f);
            m /= f;
        }
    // a lone radix-2 pass does little work per LDS round trip: 16 x 2 -> 8 x 4,
    // 8 x 2 -> 4 x 4
    auto two = std::find(rad.begin(), rad.end(), 2);
    auto big = std::find(rad.begin(), rad.end(), maxr);
    if (two != rad.end() && big != rad.end()) {
        *big /= 2;
        *two = 4;
    }
    if (m != 1 || rad.empty() || (int)rad.size() > COL_MAXP)
        return false;
    std::sort(rad.begin(), rad.end(), [](int a, int b) { return a > b; });
    return true;
}

// Per-pass twiddle tables w_L^(q j) (computed in long double, stored in the plan's
// precision) and the position of every frequency after the decimation-in-frequency
// passes (frequency k = q0 + r0 (q1 + r1 (q2 + ...)) sits at sum_i q_i s_i,
// s_i = n / (r0 ... ri)).
int setup_colfft(gsht_plan *p, ColFFT &f, int n, hipStream_t s)
{
    std::vector<int> rad;
    if (!col_radices(n, rad, col_maxr(p)))
        return fail(GSHT_EINVAL, "length %d cannot run as an in-LDS transform", n);
    f.n = n;
    f.npass = (int)rad.size();
    f.psh = p->lds_psh;
    const long double twopi = 6.283185307179586476925286766559005768L;
    std::vector<long double> re, im;
    int L = n;
    for (int i = 0; i < f.npass; ++i) {
        const int r = rad[i], st = L / r;
        f.radix[i] = r;
        f.twoff[i] = (int)re.size();
        for (int j = 0; j < st; ++j)
            for (int q = 1; q < r; ++q) {
                const long double ang = twopi * (long double)(q * j) / (long double)L;
                re.push_back(cosl(ang));
                im.push_back(-sinl(ang));
            }
        L = st;
    }
    std::vector<int32_t> perm((size_t)n);
    for (int k = 0; k < n; ++k) {
        long rest = k, stride = n, pos = 0;
        for (int i = 0; i < f.npass; ++i) {
            stride /= rad[i];
            pos += (rest % rad[i]) * stride;
            rest /= rad[i];
        }
        perm[(size_t)k] = (int32_t)pos;
    }
    const size_t nt = std::max<size_t>(re.size(), 1);
    int rc;
    void *dtw = nullptr;
    int32_t *dperm = nullptr;
    if (p->prec == GSHT_F64) {
        std::vector<double2> t(nt);
        for (size_t i = 0; i < re.size(); ++i)
            t[i] = make_double2((double)re[i], (double)im[i]);
        if ((rc = dev_alloc(p, &dtw, sizeof(double2) * nt)) != GSHT_OK) return rc;
        HIP_TRY(hipMemcpyAsync(dtw, t.data(), sizeof(double2) * nt, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        std::vector<float2> t(nt);
        for (size_t i = 0; i < re.size(); ++i)
            t[i] = make_float2((float)re[i], (float)im[i]);
        if ((rc = dev_alloc(p, &dtw, sizeof(float2) * nt)) != GSHT_OK) return rc;
        HIP_TRY(hipMemcpyAsync(dtw, t.data(), sizeof(float2) * nt, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if ((rc = dev_alloc(p, &dperm, sizeof(int32_t) * (size_t)n)) != GSHT_OK) return rc;
    HIP_TRY(hipMemcpyAsync(dperm, perm.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    f.tw = dtw;
    f.perm = dperm;
    return GSHT_OK;
}

// exp(-2 pi i k / n), k < n, in the plan precision.
int make_twist(gsht_plan *p, void **out, int n, hipStream_t s)
{
    const long double twopi = 6.283185307179586476925286766559005768L;
    int rc;
    if (p->prec == GSHT_F64) {
        std::vector<double2> t((size_t)n);
        for (int k = 0; k < n; ++k) {
            const long double ang = twopi * (long double)k / (long double)n;
            t[(size_t)k] = make_double2((double)cosl(ang), (double)-sinl(ang));
        }
        if ((rc = dev_alloc(p, out, sizeof(double2) * (size_t)n)) != GSHT_OK) return rc;
        HIP_TRY(hipMemcpyAsync(*out, t.data(), sizeof(double2) * (size_t)n, hipMemcpyHostToDevice, s));
    } else {
        std::vector<float2> t((size_t)n);
        for (int k = 0; k < n; ++k) {
            const long double ang = twopi * (long double)k / (long double)n;
            t[(size_t)k] = make_float2((float)cosl(ang), (float)-sinl(ang));
        }
        if ((rc = dev_alloc(p, out, sizeof(float2) * (size_t)n)) != GSHT_OK) return rc;
        HIP_TRY(hipMemcpyAsync(*out, t.data(), sizeof(float2) * (size_t)n, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return GSHT_OK;
}

// Smallest epsilon at which FP64 plans spread in the fast fixed-point form.
constexpr double kSpreadFastEps = 1e-10;

// Default LDS padding shift of the in-LDS transforms.
constexpr int kLdsPadShift = 4;

// Per-column FFT stage: fuse as much as fits in one workgroup's LDS.  The
// environment variable GSHT_COLUMN_MODE (0, 1, 2) forces a mode for testing.
int setup_columns(gsht_plan *p, hipStream_t s)
{
    int dev = 0, maxsh = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t lim = std::min((size_t)maxsh, COL_MAX_BYTES), cs = csize(p->prec);
    // LDS padding of the in-LDS transforms: one slot per 2^psh elements (GSHT_LDS_PAD
    // sets psh for testing; 0 turns the padding off)
    p->lds_psh = kLdsPadShift;
    if (const char *pe = getenv("GSHT_LDS_PAD")) {
        const int v = atoi(pe);
        if (v != 0 && (v < 2 || v > 30))
            return fail(GSHT_EINVAL, "GSHT_LDS_PAD=%s is not 0 or in 2..30", pe);
        p->lds_psh = v == 0 ? 31 : v;
    }
    const int psh = p->lds_psh;
    std::vector<int> rad;
    const int nh = p->n1 / 2;
    const bool fit_d = (size_t)lds_pad_n(p->nd, psh) * cs <= lim && col_radices(p->nd, rad, col_maxr(p));
    const bool fit_2 = fit_d && p->n1 % 2 == 0 && nh > p->lmax &&
                       (size_t)lds_pad_n(std::max(p->nd, nh), psh) * cs <= lim &&
                       std::max(p->nd, nh) <= column_half_maxn(p->prec) && col_radices(nh, rad, col_maxr(p));
    int mode = fit_2 ? 2 : fit_d ? 1 : 0;
    const char *e = getenv("GSHT_COLUMN_MODE");
    if (e) {
        const int want = atoi(e);
        if (want < 0 || want > 2 || (want == 2 && !fit_2) || (want == 1 && !fit_d))
            return fail(GSHT_EINVAL, "GSHT_COLUMN_MODE=%s is not possible for this plan", e);
        mode = want;
    }
    // the runtime may refuse the LDS size: then fall back to the next mode
    for (; mode > 0; --mode) {
        p->colmode = mode;
        const hipError_t he = column_set_lds(*p);
        if (he == hipSuccess)
            break;
        (void)hipGetLastError();
        if (e)
            return fail(GSHT_EHIP, "column stage LDS size refused: %s", hipGetErrorString(he));
    }
    p->colmode = mode;
    int rc;
    if (mode >= 1 && (rc = setup_colfft(p, p->cf_d, p->nd, s)) != GSHT_OK) return rc;
    if (mode == 2) {
        if ((rc = setup_colfft(p, p->cf_h, nh, s)) != GSHT_OK) return rc;
        // twist factors exp(-2 pi i k / n1) between the even and odd output rows
        const long double twopi = 6.283185307179586476925286766559005768L;
        const size_t n1 = (size_t)p->n1;
        if (p->prec == GSHT_F64) {
            std::vector<double2> t(n1);
            for (size_t k = 0; k < n1; ++k) {
                const long double ang = twopi * (long double)k / (long double)n1;
                t[k] = make_double2((double)cosl(ang), (double)-sinl(ang));
            }
            if ((rc = dev_alloc(p, &p->twist, sizeof(double2) * n1)) != GSHT_OK) return rc;
            HIP_TRY(hipMemcpyAsync(p->twist, t.data(), sizeof(double2) * n1, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        } else {
            std::vector<float2> t(n1);
            for (size_t k = 0; k < n1; ++k) {
                const long double ang = twopi * (long double)k / (long double)n1;
                t[k] = make_float2((float)cosl(ang), (float)-sinl(ang));
            }
            if ((rc = dev_alloc(p, &p->twist, sizeof(float2) * n1)) != GSHT_OK) return rc;
            HIP_TRY(hipMemcpyAsync(p->twist, t.data(), sizeof(float2) * n1, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }
    return GSHT_OK;
}

// Opt-in timing of the plan-creation phases (GSHT_PLAN_TRACE=1: one line per phase on
// stderr; the stream is synchronised at each mark, so traced creation is slower).
struct PlanTrace {
    bool on;
    hipStream_t s;
    std::chrono::steady_clock::time_point t;
    explicit PlanTrace(hipStream_t s_) : s(s_), t(std::chrono::steady_clock::now())
    {
        const char *e = getenv("GSHT_PLAN_TRACE");
        on = e && atoi(e) != 0;
    }
    void mark(const char *what)
    {
        if (!on)
            return;
        (void)hipStreamSynchronize(s);
        const auto now = std::chrono::steady_clock::now();
        fprintf(stderr, "gsht plan: %-18s %9.3f ms\n", what,
                std::chrono::duration<double, std::milli>(now - t).count());
        t = now;
    }
};

int plan_create_impl(gsht_plan **out, int lmax, int mmax, int spin, const double *theta,
                     const double *phi, int64_t npts, double eps, int prec, hipStream_t s,
                     int es_set = 0, int tile = 0)
{
    PlanTrace tr(s);
    int rc;
    gsht_plan *p = new gsht_plan();
    p->es_set = es_set;
    p->lmax = lmax;
    p->mmax = mmax;
    p->spin = spin;
    p->npts = npts;
    p->npts_cap = npts;
    p->eps = eps;
    p->prec = prec;
    p->tile_req = tile;
    // FP64 spreading: the fast fixed-point form where its rounding (relative 2^-50 of
    // a chunk's value bound per contribution) stays far below epsilon;
    // GSHT_SPREAD_QUANT=exact|fast forces a form for testing
    p->spread_fast = prec == GSHT_F64 && eps >= kSpreadFastEps;
    if (const char *q = getenv("GSHT_SPREAD_QUANT"))
        p->spread_fast = prec == GSHT_F64 && strcmp(q, "fast") == 0;
    choose_sizes(p);
    if (p->w == 0) {
        const double sg = kEs[es_set].sigma;
        delete p;
        return fail(GSHT_EUNSUPPORTED,
                    "epsilon %g is not reachable at oversampling %.2f with kernel supports up to %d",
                    eps, sg, prec == GSHT_F64 ? 16 : 8);
    }
    {
        // tile edge: the colour-ordered spreading needs patches (tile + w - 1 cells) that
        // reach at most one tile beyond their own, and each patch (16 bytes per cell in
        // FP64, 8 in FP32) must fit a workgroup's LDS beside the spreading's staging
        const int t = p->t1, pe = t + p->w - 1;
        const size_t patch = (size_t)pe * pe * (prec == GSHT_F64 ? 16 : 8) + SPREAD_STAGE_BYTES;
        if (t < 16 || t > 128 || t < p->w - 1 || patch > COL_MAX_BYTES) {
            delete p;
            return fail(GSHT_EINVAL, "tile edge %d is not possible with kernel support %d "
                                     "(16..128 cells, at least w - 1, patch of %zu bytes within "
                                     "the %zu of LDS)", t, p->w, patch, COL_MAX_BYTES);
        }
    }
    const size_t cs = csize(prec), rs = cs / 2;
    const size_t gcols = spin ? (size_t)p->n2 : (size_t)p->n2 / 2 + 1;
    // workspace estimate (before allocating anything large)
    int64_t ws = 0;
    ws += (int64_t)p->nalm * (16 + 8 + 2 * 16 * p->ncomp);   // ab, norm, uprep, acc
    ws += (int64_t)p->ncol * p->nd * cs + (int64_t)p->ncol * p->n1 * cs;
    ws += (int64_t)p->nrows * gcols * cs + (spin ? 0 : (int64_t)p->nrows * p->n2 * rs);
    ws += npts * (16 + 4) + (p->ntiles + 1) * 4;
    p->workspace_bytes = ws;
    if (ws > workspace_cap()) {
        delete p;
        return fail(GSHT_ENOMEM, "workspace of %lld bytes exceeds GSHT_MAX_WORKSPACE_BYTES",
                    (long long)ws);
    }
    std::call_once(g_fft_once, []() { rocfft_setup(); });
    tr.mark("sizes");
    if ((rc = setup_legendre(p, s, true)) != GSHT_OK) { free_plan(p); return rc; }
    tr.mark("legendre tables");
    if ((rc = dev_alloc(p, &p->D, (size_t)p->ncol * p->nd * cs)) != GSHT_OK) { free_plan(p); return rc; }
    if ((rc = dev_alloc(p, &p->E, (size_t)p->ncol * p->n1 * cs)) != GSHT_OK) { free_plan(p); return rc; }
    if ((rc = dev_alloc(p, &p->G, (size_t)p->nrows * gcols * cs)) != GSHT_OK) { free_plan(p); return rc; }
    if (!spin && (rc = dev_alloc(p, &p->g, (size_t)p->nrows * p->n2 * rs)) != GSHT_OK) { free_plan(p); return rc; }
    if ((rc = dev_alloc(p, &p->sth, sizeof(double) * (size_t)std::max<int64_t>(npts, 1))) != GSHT_OK) { free_plan(p); return rc; }
    if ((rc = dev_alloc(p, &p->sph, sizeof(double) * (size_t)std::max<int64_t>(npts, 1))) != GSHT_OK) { free_plan(p); return rc; }
    if ((rc = dev_alloc(p, &p->perm, sizeof(int32_t) * (size_t)std::max<int64_t>(npts, 1))) != GSHT_OK) { free_plan(p); return rc; }
    if ((rc = dev_alloc(p, &p->tile_start, sizeof(int32_t) * (size_t)(p->ntiles + 1))) != GSHT_OK) { free_plan(p); return rc; }
    tr.mark("allocations");
    {
        int64_t ninv = 0;
        hipError_t e = run_binsort(*p, theta, phi, s, &ninv);
        if (e != hipSuccess) {
            free_plan(p);
            return fail(GSHT_EHIP, "bin sort failed: %s", hipGetErrorString(e));
        }
        if (ninv > 0) {
            free_plan(p);
            return fail(GSHT_EINVAL, "%lld point(s) have theta outside [0, pi] or non-finite phi",
                        (long long)ninv);
        }
        tr.mark("bin sort");
        e = build_tile_colors(*p, s);
        if (e != hipSuccess) {
            free_plan(p);
            return fail(GSHT_EHIP, "tile colouring failed: %s", hipGetErrorString(e));
        }
        tr.mark("tile colours");
        p->points_ok = true;
    }
    // per-column stage, then the rocFFT plans it leaves to rocFFT
    if (p->prec == GSHT_F64) {  // interior-tap weight polynomials (GSHT_ES_POLY=0: off)
        const char *ep = getenv("GSHT_ES_POLY");
        std::vector<double> coef;
        if (!(ep && atoi(ep) == 0) && es_poly_fit(p->w, p->beta, coef)) {
            if ((rc = dev_alloc(p, &p->es_poly, sizeof(double) * coef.size())) != GSHT_OK) {
                free_plan(p);
                return rc;
            }
            const hipError_t he = hipMemcpy(p->es_poly, coef.data(), sizeof(double) * coef.size(),
                                            hipMemcpyHostToDevice);
            if (he != hipSuccess) {
                free_plan(p);
                return fail(GSHT_EHIP, "copying the kernel polynomials failed: %s",
                            hipGetErrorString(he));
            }
        }
    }
    tr.mark("kernel polynomials");
    if ((rc = setup_columns(p, s)) != GSHT_OK) { free_plan(p); return rc; }
    tr.mark("column setup");
    const size_t nd = p->nd, n1 = p->n1, n2 = p->n2;
    rc = GSHT_OK;
    if (p->colmode == 0) {
        rc = make_fft(p->fD_fwd, rocfft_transform_type_complex_forward, rocfft_placement_inplace, prec, nd, p->ncol);
        if (rc == GSHT_OK) rc = make_fft(p->fD_inv, rocfft_transform_type_complex_inverse, rocfft_placement_inplace, prec, nd, p->ncol);
    }
    if (rc == GSHT_OK && p->colmode < 2) {
        rc = make_fft(p->fT_inv, rocfft_transform_type_complex_inverse, rocfft_placement_inplace, prec, n1, p->ncol);
        if (rc == GSHT_OK) rc = make_fft(p->fT_fwd, rocfft_transform_type_complex_forward, rocfft_placement_inplace, prec, n1, p->ncol);
    }
    if (rc == GSHT_OK) {
        if (spin) {
            rc = make_fft(p->fP_inv, rocfft_transform_type_complex_inverse, rocfft_placement_inplace, prec, n2, p->nrows);
            if (rc == GSHT_OK) rc = make_fft(p->fP_fwd, rocfft_transform_type_complex_forward, rocfft_placement_inplace, prec, n2, p->nrows);
        } else {
            rc = make_fft(p->fP_inv, rocfft_transform_type_real_inverse, rocfft_placement_notinplace, prec, n2, p->nrows);
            if (rc == GSHT_OK) rc = make_fft(p->fP_fwd, rocfft_transform_type_real_forward, rocfft_placement_notinplace, prec, n2, p->nrows);
        }
    }
    if (rc != GSHT_OK) {
        free_plan(p);
        return rc;
    }
    size_t wb = 0;
    for (FFTPlan *f : {&p->fD_fwd, &p->fD_inv, &p->fT_inv, &p->fT_fwd, &p->fP_inv, &p->fP_fwd})
        wb = std::max(wb, f->work_bytes);
    if (wb) {
        if ((rc = dev_alloc(p, &p->fftwork, wb)) != GSHT_OK) { free_plan(p); return rc; }
        p->fftwork_bytes = wb;
    }
    p->workspace_bytes += (int64_t)wb;
    tr.mark("library FFT plans");
    *out = p;
    return ok();
}

// ---- profiling ----------------------------------------------------------------

struct StageScope {
    gsht_plan *p;
    int st;
    hipStream_t s;
    StageScope(gsht_plan *p_, int st_, hipStream_t s_) : p(p_), st(st_), s(s_)
    {
        if (!p->profiling)
            return;
        if (p->ev_pending[st]) {  // fold in the previous call's interval first
            float ms = 0;
            (void)hipEventSynchronize(p->ev[2 * st + 1]);
            if (hipEventElapsedTime(&ms, p->ev[2 * st], p->ev[2 * st + 1]) == hipSuccess) {
                p->st_ms[st] += ms;
                p->st_count[st] += 1;
            }
            p->ev_pending[st] = 0;
        }
        (void)hipEventRecord(p->ev[2 * st], s);
    }
    ~StageScope()
    {
        if (!p->profiling)
            return;
        (void)hipEventRecord(p->ev[2 * st + 1], s);
        p->ev_pending[st] = 1;
    }
};

#define STAGE(st) StageScope stage_scope_##st(p, st, s)

int check_launch(hipError_t e, const char *what)
{
    if (e != hipSuccess)
        return fail(GSHT_EHIP, "%s: %s", what, hipGetErrorString(e));
    return GSHT_OK;
}

// Transforms need a plan whose last bin sort and tile colouring completed.
int need_points(const gsht_plan *p)
{
    if (!p->points_ok)
        return fail(GSHT_EINVAL, "the plan has no valid points (its last gsht_plan_set_points "
                                 "failed); give it valid points first");
    return GSHT_OK;
}

#define RUN(stage, expr)                                                                       \
    do {                                                                                       \
        STAGE(stage);                                                                          \
        int rc_ = check_launch((expr), #expr);                                                 \
        if (rc_ != GSHT_OK)                                                                    \
            return rc_;                                                                        \
    } while (0)

#define RUNFFT(stage, expr)                                                                    \
    do {                                                                                       \
        STAGE(stage);                                                                          \
        int rc_ = (expr);                                                                      \
        if (rc_ != GSHT_OK)                                                                    \
            return rc_;                                                                        \
    } while (0)

int plan_synth_from_D(gsht_plan *p, hipStream_t s);

// Synthesis up to the oversampled grid (G, or g for spin 0), before interpolation.
int plan_synth_grid(gsht_plan *p, const void *alm, double mscale, hipStream_t s,
                    bool grad = false)
{
    RUN(ST_PREP, launch_prep_alm(*p, alm, mscale, grad, s));
    RUN(ST_LEG_SYNTH, launch_leg_synth(*p, p->D, grad, s));
    return plan_synth_from_D(p, s);
}

// Doubled columns D -> oversampled grid.
int plan_synth_from_D(gsht_plan *p, hipStream_t s)
{
    if (p->colmode == 0) {
        RUNFFT(ST_FFT_D_FWD, run_fft(p->fD_fwd, p->D, nullptr, p->fftwork, p->fftwork_bytes, s));
        RUN(ST_DECONV_FWD, launch_deconv_fwd(*p, s));
    } else {
        RUN(ST_COLUMN_FWD, launch_column_fwd(*p, s));
    }
    if (p->colmode < 2)
        RUNFFT(ST_FFT_THETA_INV, run_fft(p->fT_inv, p->E, nullptr, p->fftwork, p->fftwork_bytes, s));
    RUN(ST_TRANSPOSE_FWD, launch_transpose_fwd(*p, s));
    if (p->spin)
        RUNFFT(ST_FFT_PHI_INV, run_fft(p->fP_inv, p->G, nullptr, p->fftwork, p->fftwork_bytes, s));
    else
        RUNFFT(ST_FFT_PHI_INV, run_fft(p->fP_inv, p->G, p->g, p->fftwork, p->fftwork_bytes, s));
    return ok();
}

int plan_synth_impl(gsht_plan *p, const void *alm, void *map, hipStream_t s, double mscale = 1.0,
                    bool grad = false)
{
    int rc = need_points(p);
    if (rc != GSHT_OK)
        return rc;
    rc = plan_synth_grid(p, alm, mscale, s, grad);
    if (rc != GSHT_OK)
        return rc;
    RUN(ST_INTERP, launch_interp(*p, map, s));
    return ok();
}

// Synthesis with the map's derivatives along theta and phi (or, with gin, their
// products with a map gradient summed over components).
int plan_deriv_impl(gsht_plan *p, const void *alm, void *map, void *dth, void *dph,
                    const void *gin, double *gth, double *gph, hipStream_t s)
{
    int rc = need_points(p);
    if (rc != GSHT_OK)
        return rc;
    rc = plan_synth_grid(p, alm, 1.0, s);
    if (rc != GSHT_OK)
        return rc;
    RUN(ST_INTERP_DERIV, launch_interp_deriv(*p, map, dth, dph, gin, gth, gph, s));
    return ok();
}

// Adjoint from the map down to the doubled columns D (before the Legendre step).
int plan_adjoint_to_D(gsht_plan *p, const void *map, hipStream_t s)
{
    const int rc = need_points(p);
    if (rc != GSHT_OK)
        return rc;
    const size_t cs = csize(p->prec);
    if (p->spin)
        RUN(ST_ZERO_GRID, launch_zero(p->G, (size_t)p->nrows * p->n2 * cs, s));
    else
        RUN(ST_ZERO_GRID, launch_zero(p->g, (size_t)p->nrows * p->n2 * (cs / 2), s));
    RUN(ST_SPREAD, launch_spread(*p, map, s));
    if (p->spin)
        RUNFFT(ST_FFT_PHI_FWD, run_fft(p->fP_fwd, p->G, nullptr, p->fftwork, p->fftwork_bytes, s));
    else
        RUNFFT(ST_FFT_PHI_FWD, run_fft(p->fP_fwd, p->g, p->G, p->fftwork, p->fftwork_bytes, s));
    RUN(ST_TRANSPOSE_ADJ, launch_transpose_adj(*p, s));
    if (p->colmode < 2)
        RUNFFT(ST_FFT_THETA_FWD, run_fft(p->fT_fwd, p->E, nullptr, p->fftwork, p->fftwork_bytes, s));
    if (p->colmode == 0) {
        RUN(ST_DECONV_ADJ, launch_deconv_adj(*p, s));
        RUNFFT(ST_FFT_D_INV, run_fft(p->fD_inv, p->D, nullptr, p->fftwork, p->fftwork_bytes, s));
    } else {
        RUN(ST_COLUMN_ADJ, launch_column_adj(*p, s));
    }
    return ok();
}

int plan_adjoint_impl(gsht_plan *p, const void *map, void *alm, hipStream_t s,
                      double mscale = 1.0, bool grad = false)
{
    const int rc = plan_adjoint_to_D(p, map, s);
    if (rc != GSHT_OK)
        return rc;
    RUN(ST_LEG_ADJ, launch_leg_adjoint(*p, p->D, grad, s));
    RUN(ST_FINALIZE, launch_leg_finalize(*p, alm, mscale, grad, s));
    return ok();
}

const char *kStageNames[ST_COUNT] = {
    "prep_alm",     "legendre_synth", "fft_doubled_fwd", "deconv_fwd", "fft_theta_inv",
    "transpose_fwd", "fft_phi_inv",   "interp",          "zero_grid",  "spread",
    "fft_phi_fwd",  "transpose_adj",  "fft_theta_fwd",   "deconv_adj", "fft_doubled_inv",
    "legendre_adj", "finalize",       "column_fwd",      "column_adj", "interp_deriv"};

}  // namespace

extern "C" {

const char *gsht_last_error(void) { return g_last_error.c_str(); }

int gsht_plan_create(gsht_plan **p, int lmax, int mmax, int spin, const double *theta,
                     const double *phi, int64_t npts, double epsilon, gsht_precision prec,
                     void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan output pointer is NULL");
    *p = nullptr;
    int rc = check_common(lmax, mmax, spin, npts, epsilon, (int)prec);
    if (rc != GSHT_OK)
        return rc;
    if (npts > 0 && (!theta || !phi))
        return fail(GSHT_EINVAL, "theta/phi must not be NULL when npts > 0");
    return plan_create_impl(p, lmax, mmax, spin, theta, phi, npts, epsilon, (int)prec,
                            (hipStream_t)hip_stream);
}

int gsht_plan_create_sigma(gsht_plan **p, int lmax, int mmax, int spin, const double *theta,
                           const double *phi, int64_t npts, double epsilon, gsht_precision prec,
                           double sigma, void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan output pointer is NULL");
    *p = nullptr;
    const int set = es_set_of(sigma);
    if (set < 0)
        return fail(GSHT_EINVAL, "sigma must be 2, 1.5 or 1.25, got %g", sigma);
    int rc = check_common(lmax, mmax, spin, npts, epsilon, (int)prec);
    if (rc != GSHT_OK)
        return rc;
    if (npts > 0 && (!theta || !phi))
        return fail(GSHT_EINVAL, "theta/phi must not be NULL when npts > 0");
    return plan_create_impl(p, lmax, mmax, spin, theta, phi, npts, epsilon, (int)prec,
                            (hipStream_t)hip_stream, set);
}

int gsht_plan_set_points(gsht_plan *p, const double *theta, const double *phi, int64_t npts,
                         void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (npts < 0 || npts > p->npts_cap)
        return fail(GSHT_EINVAL, "npts must be in [0, %lld] (the plan's capacity), got %lld",
                    (long long)p->npts_cap, (long long)npts);
    if (npts > 0 && (!theta || !phi))
        return fail(GSHT_EINVAL, "theta/phi must not be NULL when npts > 0");
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(hipStreamSynchronize(s));  // earlier transforms may still read the old sort
    // the chunk list, tile items and colours of the previous sort are rebuilt; until
    // that has completed the plan refuses every transform
    p->points_ok = false;
    p->ncolors = 0;
    p->nchunks = 0;
    for (void **q : {(void **)&p->chunks, (void **)&p->tile_items}) {
        if (!*q)
            continue;
        auto it = std::find(p->allocations.begin(), p->allocations.end(), *q);
        if (it != p->allocations.end())
            p->allocations.erase(it);
        (void)hipFree(*q);
        *q = nullptr;
    }
    p->npts = npts;
    p->nchunks = 0;
    int64_t ninv = 0;
    hipError_t e = run_binsort(*p, theta, phi, s, &ninv);
    if (e != hipSuccess)
        return fail(GSHT_EHIP, "bin sort failed: %s", hipGetErrorString(e));
    if (ninv > 0)
        return fail(GSHT_EINVAL, "%lld point(s) have theta outside [0, pi] or non-finite phi "
                                 "(the plan must get valid points before its next use)",
                    (long long)ninv);
    e = build_tile_colors(*p, s);
    if (e != hipSuccess)
        return fail(GSHT_EHIP, "tile colouring failed: %s", hipGetErrorString(e));
    p->points_ok = true;
    return ok();
}

int gsht_plan_synth(gsht_plan *p, const void *alm, void *map, void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (!alm || (!map && p->npts > 0))
        return fail(GSHT_EINVAL, "alm/map must not be NULL");
    return plan_synth_impl(p, alm, map, (hipStream_t)hip_stream);
}

int gsht_plan_adjoint(gsht_plan *p, const void *map, void *alm, void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (!alm || (!map && p->npts > 0))
        return fail(GSHT_EINVAL, "alm/map must not be NULL");
    return plan_adjoint_impl(p, map, alm, (hipStream_t)hip_stream);
}

int gsht_plan_create_tuned(gsht_plan **p, int lmax, int mmax, int spin, const double *theta,
                           const double *phi, int64_t npts, double epsilon, gsht_precision prec,
                           void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan output pointer is NULL");
    *p = nullptr;
    int rc = check_common(lmax, mmax, spin, npts, epsilon, (int)prec);
    if (rc != GSHT_OK)
        return rc;
    if (npts > 0 && (!theta || !phi))
        return fail(GSHT_EINVAL, "theta/phi must not be NULL when npts > 0");
    hipStream_t s = (hipStream_t)hip_stream;
    const int ncomp = spin ? 2 : 1;
    const size_t cs = csize((int)prec);
    const size_t alm_bytes = cs * ncomp * (size_t)((int64_t)(mmax + 1) * (lmax + 1) -
                                                   (int64_t)mmax * (mmax + 1) / 2);
    const size_t map_bytes = cs / 2 * ncomp * (size_t)std::max<int64_t>(npts, 1);
    void *alm = nullptr, *map = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    gsht_plan *best = nullptr;
    float best_ms = -1.0f;
    auto cleanup = [&]() {
        if (alm) (void)hipFree(alm);
        if (map) (void)hipFree(map);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc(&alm, alm_bytes) != hipSuccess || hipMalloc(&map, map_bytes) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(GSHT_ENOMEM, "tuning buffers could not be allocated");
    }
    // coefficient values do not change the work; the map must be non-zero, or the
    // spreading step would skip every chunk
    if (launch_zero(alm, alm_bytes, s) != hipSuccess ||
        launch_fill_real(map, 1.0, (int64_t)(map_bytes / (cs / 2)), (int)prec, s) != hipSuccess) {
        cleanup();
        return fail(GSHT_EHIP, "preparing the tuning buffers failed");
    }
    const int tiles[3] = {32, 48, 64};
    for (int cand = 0; cand < 3 * kNumEs; ++cand) {
        const int set = cand / 3, tile = tiles[cand % 3];
        gsht_plan *c = nullptr;
        rc = plan_create_impl(&c, lmax, mmax, spin, theta, phi, npts, epsilon, (int)prec, s, set,
                              tile);
        if (rc != GSHT_OK) {
            if (cand == 0) {  // the default setting must build
                cleanup();
                return rc;
            }
            continue;  // not reachable at this sigma or tile, or no room for a second plan
        }
        // one synthesis + adjoint to warm up, then the best of two
        float t = -1.0f;
        bool good = plan_synth_impl(c, alm, map, s) == GSHT_OK &&
                    plan_adjoint_impl(c, map, alm, s) == GSHT_OK;
        for (int rep = 0; good && rep < 2; ++rep) {
            float ms = 0;
            good = hipEventRecord(e0, s) == hipSuccess && plan_synth_impl(c, alm, map, s) == GSHT_OK &&
                   plan_adjoint_impl(c, map, alm, s) == GSHT_OK &&
                   hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                   hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (good)
                t = (t < 0 || ms < t) ? ms : t;
        }
        if (!good) {
            free_plan(c);
            if (best)
                free_plan(best);
            cleanup();
            return fail(GSHT_EHIP, "timing the candidate plan at sigma %.2f, tile %d failed",
                        kEs[set].sigma, tile);
        }
        if (best_ms < 0 || t < best_ms) {
            if (best)
                free_plan(best);
            best = c;
            best_ms = t;
        } else {
            free_plan(c);
        }
    }
    cleanup();
    *p = best;
    return ok();
}

int gsht_plan_autotune(gsht_plan *p, void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (!p->D || !p->uprep)
        return fail(GSHT_EINVAL, "plan has no Legendre buffers");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nck1 = (p->npairs + 63) / 64;  // chunks at one slice per wave (the most)
    int32_t *ls = nullptr, *la = nullptr;
    int rc;
    if ((rc = dev_alloc(p, &ls, sizeof(int32_t) * (size_t)(p->mmax + 1) * nck1)) != GSHT_OK)
        return rc;
    if ((rc = dev_alloc(p, &la, sizeof(int32_t) * (size_t)(p->mmax + 1) * nck1)) != GSHT_OK)
        return rc;
    HIP_TRY(launch_zero(p->uprep, sizeof(double) * 2 * p->ncomp * (size_t)p->nalm, s));
    HIP_TRY(launch_zero(p->D, (size_t)p->ncol * p->nd * csize(p->prec), s));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GSHT_EHIP, "hipEventCreate failed");
    }
    auto set_shape = [&](int sr, int ar, int ab) {
        p->syn_r = sr;
        p->adj_r = ar;
        p->adj_b = ab;
        p->syn_nchunk = (p->npairs + 64 * sr - 1) / (64 * sr);
        p->adj_nchunk = (p->npairs + 64 * ar - 1) / (64 * ar);
        p->leg.lfirst_syn = ls;
        p->leg.lfirst_adj = la;
        return launch_leg_live(*p, s);
    };
    // best of two runs of one launch, in ms (negative on a launch error)
    auto time_ms = [&](auto launch) {
        float best = -1.0f;
        for (int rep = 0; rep < 2; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess || launch() != hipSuccess ||
                hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return -1.0f;
            float ms = 0;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                return -1.0f;
            best = (best < 0 || ms < best) ? ms : best;
        }
        return best;
    };
    const int ar0 = p->adj_r, ab0 = p->adj_b;
    int best_sr = p->syn_r;
    float best_t = -1.0f;
    for (int sr : {1, 2, 4}) {
        if (set_shape(sr, ar0, ab0) != hipSuccess)
            break;
        const float t = time_ms([&] { return launch_leg_synth(*p, p->D, false, s); });
        if (t >= 0 && (best_t < 0 || t < best_t)) {
            best_t = t;
            best_sr = sr;
        }
    }
    int best_ar = ar0, best_ab = ab0;
    best_t = -1.0f;
    const int shapes[7][2] = {{1, 8}, {2, 8}, {2, 4}, {4, 4}, {3, 8}, {3, 4}, {4, 8}};
    for (const auto &sh : shapes) {
        if (set_shape(best_sr, sh[0], sh[1]) != hipSuccess)
            break;
        const float t = time_ms([&] { return launch_leg_adjoint(*p, p->D, false, s); });
        if (t >= 0 && (best_t < 0 || t < best_t)) {
            best_t = t;
            best_ar = sh[0];
            best_ab = sh[1];
        }
    }
    const hipError_t e = set_shape(best_sr, best_ar, best_ab);
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess)
        return fail(GSHT_EHIP, "autotune: %s", hipGetErrorString(e));
    return ok();
}

// The matrix-core Legendre step serves FP32 plans (epsilon >= 1e-5) with lmax <= 8192,
// where every Legendre value times 2^7 fits FP16 (|p_l| <= sqrt((2 l + 1) / 4 pi) / N_l
// with N_l >= 0.14); GSHT_MANY_MFMA=0 turns it off.
static bool use_mfma(const gsht_plan *p)
{
    if (p->prec != GSHT_F32 || p->lmax > 8192)
        return false;
    const char *e = getenv("GSHT_MANY_MFMA");
    return !(e && atoi(e) == 0);
}

// Buffers of the matrix-core step, sized for 16 maps: tile offsets per m (16 degrees
// per block from l0 = max(m, s)), tiles, scales, doubled columns, dead-chunk table.
static int setup_mfma(gsht_plan *p, hipStream_t s)
{
    if (p->mfma_tiles)
        return GSHT_OK;
    int rc;
    std::vector<int64_t> boff((size_t)p->mmax + 1);
    int64_t nblk = 0;
    for (int m = 0; m <= p->mmax; ++m) {
        boff[(size_t)m] = nblk;
        const int l0 = std::max(m, p->spin);
        if (l0 <= p->lmax)
            nblk += (p->lmax - l0 + 16) / 16;
    }
    const size_t nt = p->spin ? 2 : 1;
    const size_t tile_bytes = (size_t)nblk * nt * 2 /* column blocks */ * 2 /* hi, lo */ * 64 * 16;
    const size_t dstride = (size_t)p->ncol * p->nd;
    const int nchunk = (p->npairs + 63) / 64;
    if ((rc = dev_alloc(p, &p->mfma_boff, sizeof(int64_t) * boff.size())) != GSHT_OK) return rc;
    if ((rc = dev_alloc(p, &p->mfma_scale, sizeof(float) * 16 * boff.size())) != GSHT_OK) return rc;
    if ((rc = dev_alloc(p, &p->mfma_live, sizeof(int32_t) * (size_t)nchunk * boff.size())) != GSHT_OK)
        return rc;
    if ((rc = dev_alloc(p, &p->Dmfma, 16 * dstride * csize(p->prec))) != GSHT_OK) return rc;
    if ((rc = dev_alloc(p, &p->mfma_tiles, tile_bytes)) != GSHT_OK) {
        p->mfma_tiles = nullptr;
        return rc;
    }
    HIP_TRY(hipMemcpyAsync(p->mfma_boff, boff.data(), sizeof(int64_t) * boff.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(launch_leg_live_r1(*p, p->mfma_live, s));
    HIP_TRY(hipStreamSynchronize(s));
    return GSHT_OK;
}

// Buffers of the matrix-core adjoint (16 maps): ring-input tiles per (m, slice, 32-ring
// step), scales, sums; the doubled columns and the dead-chunk table are shared with
// the matrix-core synthesis.
static int setup_mfma_adj(gsht_plan *p, hipStream_t s)
{
    int rc;
    if ((rc = setup_mfma(p, s)) != GSHT_OK)
        return rc;
    if (p->mfma_atiles)
        return GSHT_OK;
    const size_t nslice = (size_t)(p->npairs + 63) / 64, nm1 = (size_t)p->mmax + 1;
    const size_t nt = p->spin ? 2 : 1;
    const size_t tile_bytes = nm1 * nslice * 2 * nt * 4 /* column blocks */ * 2 * 64 * 16;
    if ((rc = dev_alloc(p, &p->mfma_ascale, sizeof(float) * 16 * nm1)) != GSHT_OK) return rc;
    if ((rc = dev_alloc(p, &p->mfma_acc, sizeof(double) * 16 * (size_t)p->nalm * 2 * p->ncomp)) !=
        GSHT_OK)
        return rc;
    if ((rc = dev_alloc(p, &p->mfma_rstate, adj_mfma_state_bytes(*p))) != GSHT_OK) return rc;
    if ((rc = dev_alloc(p, &p->mfma_atiles, tile_bytes)) != GSHT_OK) {
        p->mfma_atiles = nullptr;
        return rc;
    }
    return GSHT_OK;
}

static bool use_mfma_adj(const gsht_plan *p)
{
    int S, W;
    adj_mfma_shape(*p, S, W);
    return use_mfma(p) && W > 0;
}

int gsht_plan_adjoint_many(gsht_plan *p, int nmaps, const void *map, void *alm, void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (nmaps < 0)
        return fail(GSHT_EINVAL, "nmaps must be >= 0, got %d", nmaps);
    if (nmaps > 0 && (!alm || (!map && p->npts > 0)))
        return fail(GSHT_EINVAL, "map/alm must not be NULL");
    if (nmaps > 0 && need_points(p) != GSHT_OK)
        return GSHT_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t cs = csize(p->prec);
    const size_t astride = (size_t)p->ncomp * p->nalm * cs;
    const size_t mstride = (size_t)p->ncomp * p->npts * (cs / 2);
    const size_t dstride = (size_t)p->ncol * p->nd;
    const size_t nr = (size_t)2 * p->ncomp;
    int rc;
    const bool mfma = use_mfma_adj(p);
    for (int k = 0; k < nmaps;) {
        const char *mk = (const char *)map + (map ? k * mstride : 0);
        char *ak = (char *)alm + k * astride;
        if (mfma && nmaps - k >= 8) {
            const int nm = std::min(16, nmaps - k);
            if ((rc = setup_mfma_adj(p, s)) != GSHT_OK)
                return rc;
            for (int j = 0; j < nm; ++j) {
                void *dsave = p->D;
                p->D = (char *)p->Dmfma + j * dstride * cs;
                rc = plan_adjoint_to_D(p, mk + j * mstride, s);
                p->D = dsave;
                if (rc != GSHT_OK)
                    return rc;
            }
            RUN(ST_PREP, launch_prep_adj_mfma(*p, nm, p->Dmfma, dstride, p->mfma_atiles,
                                              p->mfma_ascale, s));
            RUN(ST_LEG_ADJ, launch_leg_adjoint_mfma(*p, nm, p->mfma_atiles, p->mfma_ascale,
                                                    p->mfma_live, p->mfma_rstate, p->mfma_acc, s));
            for (int j = 0; j < nm; ++j) {
                double *asave = p->acc;
                p->acc = p->mfma_acc + j * (size_t)p->nalm * nr;
                const hipError_t he = launch_leg_finalize(*p, ak + j * astride, 1.0, false, s);
                p->acc = asave;
                if ((rc = check_launch(he, "launch_leg_finalize")) != GSHT_OK)
                    return rc;
            }
            k += nm;
            continue;
        }
        if ((rc = plan_adjoint_impl(p, mk, ak, s)) != GSHT_OK)
            return rc;
        k += 1;
    }
    return ok();
}

int gsht_plan_synth_many(gsht_plan *p, int nmaps, const void *alm, void *map, void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (nmaps < 0)
        return fail(GSHT_EINVAL, "nmaps must be >= 0, got %d", nmaps);
    if (nmaps > 0 && (!alm || (!map && p->npts > 0)))
        return fail(GSHT_EINVAL, "alm/map must not be NULL");
    if (nmaps > 0 && need_points(p) != GSHT_OK)
        return GSHT_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t cs = csize(p->prec);
    const size_t astride = (size_t)p->ncomp * p->nalm * cs;
    const size_t mstride = (size_t)p->ncomp * p->npts * (cs / 2);
    const size_t dstride = (size_t)p->ncol * p->nd;  // complex elements per map
    int rc;
    const bool mfma = use_mfma(p);
    for (int k = 0; k < nmaps;) {
        if (mfma && nmaps - k >= 8) {  // matrix-core Legendre step, up to 16 maps
            const int nm = std::min(16, nmaps - k);
            if ((rc = setup_mfma(p, s)) != GSHT_OK)
                return rc;
            const char *ak = (const char *)alm + k * astride;
            char *mk = (char *)map + (map ? k * mstride : 0);
            RUN(ST_PREP, launch_prep_mfma(*p, ak, nm, p->mfma_boff, p->mfma_tiles, p->mfma_scale, s));
            RUN(ST_LEG_SYNTH, launch_leg_synth_mfma(*p, nm, p->mfma_tiles, p->mfma_scale,
                                                    p->mfma_boff, p->mfma_live, p->Dmfma, dstride, s));
            for (int j = 0; j < nm; ++j) {
                void *dsave = p->D;
                p->D = (char *)p->Dmfma + j * dstride * cs;
                rc = plan_synth_from_D(p, s);
                p->D = dsave;
                if (rc != GSHT_OK)
                    return rc;
                RUN(ST_INTERP, launch_interp(*p, mk + j * mstride, s));
            }
            k += nm;
            continue;
        }
        int nm = nmaps - k >= 4 ? 4 : (nmaps - k >= 2 ? 2 : 1);
        if (p->syn_r > 2)
            nm = 1;
        const char *ak = (const char *)alm + k * astride;
        char *mk = (char *)map + (map ? k * mstride : 0);
        if (nm == 1) {
            if ((rc = plan_synth_impl(p, ak, mk, s)) != GSHT_OK)
                return rc;
            k += 1;
            continue;
        }
        if (!p->umulti &&
            (rc = dev_alloc(p, &p->umulti, sizeof(double) * 4 * 2 * p->ncomp * (size_t)p->nalm)) !=
                GSHT_OK)
            return rc;
        if (!p->Dmulti && (rc = dev_alloc(p, &p->Dmulti, 4 * dstride * cs)) != GSHT_OK)
            return rc;
        RUN(ST_PREP, launch_prep_multi(*p, ak, nm, p->umulti, s));
        RUN(ST_LEG_SYNTH, launch_leg_synth_multi(*p, nm, p->umulti, p->Dmulti, dstride, s));
        for (int j = 0; j < nm; ++j) {
            void *dsave = p->D;
            p->D = (char *)p->Dmulti + j * dstride * cs;
            rc = plan_synth_from_D(p, s);
            p->D = dsave;
            if (rc != GSHT_OK)
                return rc;
            RUN(ST_INTERP, launch_interp(*p, mk + j * mstride, s));
        }
        k += nm;
    }
    return ok();
}

int gsht_plan_synth_grad(gsht_plan *p, const void *glm, void *map, void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (p->spin == 0)
        return fail(GSHT_EINVAL, "gradient-only transforms need spin > 0");
    if (!glm || (!map && p->npts > 0))
        return fail(GSHT_EINVAL, "glm/map must not be NULL");
    return plan_synth_impl(p, glm, map, (hipStream_t)hip_stream, 1.0, true);
}

int gsht_plan_adjoint_grad(gsht_plan *p, const void *map, void *glm, void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (p->spin == 0)
        return fail(GSHT_EINVAL, "gradient-only transforms need spin > 0");
    if (!glm || (!map && p->npts > 0))
        return fail(GSHT_EINVAL, "glm/map must not be NULL");
    return plan_adjoint_impl(p, map, glm, (hipStream_t)hip_stream, 1.0, true);
}

int gsht_plan_synth_deriv(gsht_plan *p, const void *alm, void *map, void *dtheta, void *dphi,
                          void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (!alm)
        return fail(GSHT_EINVAL, "alm must not be NULL");
    if (!map && !dtheta && !dphi)
        return fail(GSHT_EINVAL, "at least one of map/dtheta/dphi must be given");
    return plan_deriv_impl(p, alm, map, dtheta, dphi, nullptr, nullptr, nullptr,
                           (hipStream_t)hip_stream);
}

int gsht_plan_synth_vjp(gsht_plan *p, const void *alm, const void *gmap, void *galm,
                        double *gtheta, double *gphi, void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (!gmap && p->npts > 0)
        return fail(GSHT_EINVAL, "gmap must not be NULL");
    if ((gtheta || gphi) && !alm)
        return fail(GSHT_EINVAL, "alm is needed for position gradients");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = GSHT_OK;
    if (galm && (rc = plan_adjoint_impl(p, gmap, galm, s, 2.0)) != GSHT_OK)
        return rc;
    if (gtheta || gphi)
        rc = plan_deriv_impl(p, alm, nullptr, nullptr, nullptr, gmap, gtheta, gphi, s);
    return rc;
}

int gsht_plan_adjoint_vjp(gsht_plan *p, const void *galm, void *gmap, void *hip_stream)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (!galm || (!gmap && p->npts > 0))
        return fail(GSHT_EINVAL, "galm/gmap must not be NULL");
    return plan_synth_impl(p, galm, gmap, (hipStream_t)hip_stream, 0.5);
}

void gsht_plan_destroy(gsht_plan *p) { free_plan(p); }

// ---- batches of plans -------------------------------------------------------------

struct gsht_batch {
    std::vector<hipStream_t> streams;  // worker streams (default priority, non-blocking)
    std::vector<hipEvent_t> joins;     // one per worker stream
    hipEvent_t fork = nullptr;
};

static void free_batch(gsht_batch *b)
{
    if (!b)
        return;
    for (hipEvent_t e : b->joins)
        (void)hipEventDestroy(e);
    if (b->fork)
        (void)hipEventDestroy(b->fork);
    for (hipStream_t s : b->streams)
        (void)hipStreamDestroy(s);
    delete b;
}

int gsht_batch_create(gsht_batch **out, int nstreams)
{
    if (!out)
        return fail(GSHT_EINVAL, "batch output pointer is NULL");
    *out = nullptr;
    if (nstreams < 1 || nstreams > 16)
        return fail(GSHT_EINVAL, "nstreams must be in [1, 16], got %d", nstreams);
    gsht_batch *b = new gsht_batch();
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int i = 0; i < nstreams && e == hipSuccess; ++i) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess)
            b->streams.push_back(st);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess)
            b->joins.push_back(ev);
    }
    if (e != hipSuccess) {
        free_batch(b);
        return fail(GSHT_EHIP, "batch creation failed: %s", hipGetErrorString(e));
    }
    *out = b;
    return ok();
}

void gsht_batch_destroy(gsht_batch *b) { free_batch(b); }

// Instance i on worker stream i mod nstreams, after the work already queued on
// hip_stream; hip_stream then waits for every worker.
static int batch_run(gsht_batch *b, int n, gsht_plan *const *plans, const void *const *in,
                     void *const *out, void *hip_stream, bool adjoint)
{
    if (!b)
        return fail(GSHT_EINVAL, "batch is NULL");
    if (n < 0)
        return fail(GSHT_EINVAL, "n must be >= 0, got %d", n);
    if (n == 0)
        return ok();
    if (!plans || !in || !out)
        return fail(GSHT_EINVAL, "plans/inputs/outputs must not be NULL");
    for (int i = 0; i < n; ++i) {
        if (!plans[i])
            return fail(GSHT_EINVAL, "plan %d is NULL", i);
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i])
                return fail(GSHT_EINVAL, "plan %d appears twice in the batch (instances %d and %d "
                                         "would share its work buffers)", i, j, i);
        if (need_points(plans[i]) != GSHT_OK)
            return fail(GSHT_EINVAL, "plan %d has no valid points (its last gsht_plan_set_points "
                                     "failed)", i);
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const int ns = (int)b->streams.size();
    const int used = n < ns ? n : ns;
    HIP_TRY(hipEventRecord(b->fork, s));
    for (int k = 0; k < used; ++k)
        HIP_TRY(hipStreamWaitEvent(b->streams[(size_t)k], b->fork, 0));
    int rc = GSHT_OK;
    for (int i = 0; i < n && rc == GSHT_OK; ++i) {
        hipStream_t ws = b->streams[(size_t)(i % ns)];
        rc = adjoint ? plan_adjoint_impl(plans[i], in[i], out[i], ws)
                     : plan_synth_impl(plans[i], in[i], out[i], ws);
    }
    // join every worker that was forked, also after an error
    for (int k = 0; k < used; ++k) {
        HIP_TRY(hipEventRecord(b->joins[(size_t)k], b->streams[(size_t)k]));
        HIP_TRY(hipStreamWaitEvent(s, b->joins[(size_t)k], 0));
    }
    return rc == GSHT_OK ? ok() : rc;
}

int gsht_batch_synth(gsht_batch *b, int n, gsht_plan *const *plans, const void *const *alms,
                     void *const *maps, void *hip_stream)
{
    return batch_run(b, n, plans, alms, maps, hip_stream, false);
}

int gsht_batch_adjoint(gsht_batch *b, int n, gsht_plan *const *plans, const void *const *maps,
                       void *const *alms, void *hip_stream)
{
    return batch_run(b, n, plans, maps, alms, hip_stream, true);
}

int gsht_deflect(const double *theta, const double *phi, const void *alpha, gsht_precision prec,
                 int64_t npts, double *theta_out, double *phi_out, double *chi_out,
                 void *hip_stream)
{
    if (prec != GSHT_F64 && prec != GSHT_F32)
        return fail(GSHT_EINVAL, "unknown precision %d", (int)prec);
    if (npts < 0)
        return fail(GSHT_EINVAL, "npts must be >= 0");
    if (npts > 0 && (!theta || !phi || !alpha || !theta_out || !phi_out))
        return fail(GSHT_EINVAL, "theta/phi/alpha/theta_out/phi_out must not be NULL");
    return check_launch(launch_deflect(theta, phi, alpha, prec, npts, theta_out, phi_out, chi_out,
                                       (hipStream_t)hip_stream),
                        "deflect");
}

int gsht_deflect_vjp(const double *theta, const void *alpha, gsht_precision prec, int64_t npts,
                     const double *g_theta, const double *g_phi, const double *g_chi,
                     void *g_alpha, void *hip_stream)
{
    if (prec != GSHT_F64 && prec != GSHT_F32)
        return fail(GSHT_EINVAL, "unknown precision %d", (int)prec);
    if (npts < 0)
        return fail(GSHT_EINVAL, "npts must be >= 0");
    if (npts > 0 && (!theta || !alpha || !g_alpha))
        return fail(GSHT_EINVAL, "theta/alpha/g_alpha must not be NULL");
    return check_launch(launch_deflect_vjp(theta, alpha, prec, npts, g_theta, g_phi, g_chi, g_alpha,
                                           (hipStream_t)hip_stream),
                        "deflect_vjp");
}

int gsht_spin_phase(void *map, const double *chi, int spin, int sign, gsht_precision prec,
                    int64_t npts, void *hip_stream)
{
    if (prec != GSHT_F64 && prec != GSHT_F32)
        return fail(GSHT_EINVAL, "unknown precision %d", (int)prec);
    if (npts < 0 || (sign != 1 && sign != -1))
        return fail(GSHT_EINVAL, "npts must be >= 0 and sign +1 or -1");
    if (npts > 0 && (!map || !chi))
        return fail(GSHT_EINVAL, "map/chi must not be NULL");
    return check_launch(launch_spin_phase(map, chi, spin, sign, prec, npts,
                                          (hipStream_t)hip_stream),
                        "spin_phase");
}

int gsht_spin_phase_vjp(const void *gmap, const void *lensed, const double *chi, int spin,
                        gsht_precision prec, int64_t npts, void *g_unrot, double *g_chi,
                        void *hip_stream)
{
    if (prec != GSHT_F64 && prec != GSHT_F32)
        return fail(GSHT_EINVAL, "unknown precision %d", (int)prec);
    if (npts < 0)
        return fail(GSHT_EINVAL, "npts must be >= 0");
    if (npts > 0 && (!gmap || !chi || (g_chi && !lensed) || (!g_unrot && !g_chi)))
        return fail(GSHT_EINVAL, "gmap/chi (and lensed for g_chi) must not be NULL; "
                                 "at least one output");
    return check_launch(launch_spin_phase_vjp(gmap, lensed, chi, spin, prec, npts, g_unrot, g_chi,
                                              (hipStream_t)hip_stream),
                        "spin_phase_vjp");
}

int gsht_map_weight(const void *map_in, const double *weights, int ncomp, int64_t npts,
                    gsht_precision prec, void *map_out, void *hip_stream)
{
    if (prec != GSHT_F64 && prec != GSHT_F32)
        return fail(GSHT_EINVAL, "unknown precision %d", (int)prec);
    if (npts < 0 || ncomp < 1 || ncomp > 2)
        return fail(GSHT_EINVAL, "need npts >= 0 and ncomp in {1, 2}");
    if (npts > 0 && (!map_in || !weights || !map_out))
        return fail(GSHT_EINVAL, "map_in/weights/map_out must not be NULL");
    return check_launch(launch_map_weight(map_in, weights, ncomp, npts, prec, map_out,
                                          (hipStream_t)hip_stream),
                        "map_weight");
}

int gsht_alm_lscale(const void *alm_in, void *alm_out, int lmax, int mmax, int ncomp,
                    gsht_precision prec, void *hip_stream)
{
    if (prec != GSHT_F64 && prec != GSHT_F32)
        return fail(GSHT_EINVAL, "unknown precision %d", (int)prec);
    if (lmax < 0 || mmax < 0 || mmax > lmax || lmax > 32766 || ncomp < 1 || ncomp > 2)
        return fail(GSHT_EINVAL, "need 0 <= mmax <= lmax <= 32766 and ncomp in {1, 2}");
    if (!alm_in || !alm_out)
        return fail(GSHT_EINVAL, "alm_in/alm_out must not be NULL");
    return check_launch(launch_alm_lscale(alm_in, lmax, mmax, ncomp, 0, prec, alm_out,
                                          (hipStream_t)hip_stream),
                        "alm_lscale");
}

int gsht_alm_lfactor(const void *alm_in, void *alm_out, int lmax, int mmax, int ncomp, int kind,
                     gsht_precision prec, void *hip_stream)
{
    if (prec != GSHT_F64 && prec != GSHT_F32)
        return fail(GSHT_EINVAL, "unknown precision %d", (int)prec);
    if (lmax < 0 || mmax < 0 || mmax > lmax || lmax > 32766 || ncomp < 1 || ncomp > 2)
        return fail(GSHT_EINVAL, "need 0 <= mmax <= lmax <= 32766 and ncomp in {1, 2}");
    if (kind < 0 || kind > 2)
        return fail(GSHT_EINVAL, "kind must be 0, 1 or 2, got %d", kind);
    if (!alm_in || !alm_out)
        return fail(GSHT_EINVAL, "alm_in/alm_out must not be NULL");
    return check_launch(launch_alm_lscale(alm_in, lmax, mmax, ncomp, kind, prec, alm_out,
                                          (hipStream_t)hip_stream),
                        "alm_lfactor");
}

int gsht_magnification(const void *alpha, const void *kappa, const void *omega, const void *gamma,
                       gsht_precision prec, int64_t npts, double *det, void *hip_stream)
{
    if (prec != GSHT_F64 && prec != GSHT_F32)
        return fail(GSHT_EINVAL, "unknown precision %d", (int)prec);
    if (npts < 0)
        return fail(GSHT_EINVAL, "npts must be >= 0");
    if (npts > 0 && (!alpha || !kappa || !gamma || !det))
        return fail(GSHT_EINVAL, "alpha/kappa/gamma/det must not be NULL");
    return check_launch(launch_magnification(alpha, kappa, omega, gamma, prec, npts, det,
                                             (hipStream_t)hip_stream),
                        "magnification");
}

int gsht_synth_general(const void *alm, int lmax, int mmax, int spin, const double *theta,
                       const double *phi, int64_t npts, double epsilon, gsht_precision prec,
                       void *map, void *hip_stream)
{
    if (!alm || (!map && npts > 0))
        return fail(GSHT_EINVAL, "alm/map must not be NULL");
    gsht_plan *p = nullptr;
    int rc = gsht_plan_create(&p, lmax, mmax, spin, theta, phi, npts, epsilon, prec, hip_stream);
    if (rc != GSHT_OK)
        return rc;
    rc = plan_synth_impl(p, alm, map, (hipStream_t)hip_stream);
    free_plan(p);
    return rc;
}

int gsht_adjoint_synth_general(const void *map, int lmax, int mmax, int spin, const double *theta,
                               const double *phi, int64_t npts, double epsilon,
                               gsht_precision prec, void *alm, void *hip_stream)
{
    if (!alm || (!map && npts > 0))
        return fail(GSHT_EINVAL, "alm/map must not be NULL");
    gsht_plan *p = nullptr;
    int rc = gsht_plan_create(&p, lmax, mmax, spin, theta, phi, npts, epsilon, prec, hip_stream);
    if (rc != GSHT_OK)
        return rc;
    rc = plan_adjoint_impl(p, map, alm, (hipStream_t)hip_stream);
    free_plan(p);
    return rc;
}

int gsht_plan_get_info(const gsht_plan *p, gsht_plan_info *info)
{
    if (!p || !info)
        return fail(GSHT_EINVAL, "plan/info must not be NULL");
    info->lmax = p->lmax;
    info->mmax = p->mmax;
    info->spin = p->spin;
    info->ncomp = p->ncomp;
    info->npts = p->npts;
    info->epsilon = p->eps;
    info->precision = p->prec;
    info->ntheta = p->ntheta;
    info->ndouble = p->nd;
    info->n1 = p->n1;
    info->n2 = p->n2;
    info->w = p->w;
    info->beta = p->beta;
    info->sigma = kEs[p->es_set].sigma;
    info->nrows = p->nrows;
    info->a_min = p->a_min;
    info->tile1 = p->t1;
    info->tile2 = p->t2;
    info->ntile1 = p->nt1;
    info->ntile2 = p->nt2;
    info->nchunks = p->nchunks;
    info->workspace_bytes = p->workspace_bytes;
    info->column_mode = p->colmode;
    info->spread_colors = p->ncolors;
    info->cell_sort = p->cell_sort ? 1 : 0;
    info->syn_r = p->syn_r;
    info->adj_r = p->adj_r;
    info->adj_b = p->adj_b;
    return ok();
}

int gsht_plan_get_sort(const gsht_plan *p, int32_t *perm, int32_t *tile_start, void *hip_stream)
{
    if (!p || !perm || !tile_start)
        return fail(GSHT_EINVAL, "plan/perm/tile_start must not be NULL");
    if (need_points(p) != GSHT_OK)
        return GSHT_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    if (p->npts > 0)
        HIP_TRY(hipMemcpyAsync(perm, p->perm, sizeof(int32_t) * (size_t)p->npts,
                               hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(tile_start, p->tile_start, sizeof(int32_t) * (size_t)(p->ntiles + 1),
                           hipMemcpyDeviceToDevice, s));
    return ok();
}

int gsht_plan_set_profiling(gsht_plan *p, int on)
{
    if (!p)
        return fail(GSHT_EINVAL, "plan is NULL");
    if (on) {
        for (int i = 0; i < 2 * ST_COUNT; ++i)
            if (!p->ev[i])
                HIP_TRY(hipEventCreate(&p->ev[i]));
    }
    for (int i = 0; i < ST_COUNT; ++i) {
        p->st_ms[i] = 0;
        p->st_count[i] = 0;
        p->ev_pending[i] = 0;
    }
    p->profiling = on ? 1 : 0;
    return ok();
}

int gsht_plan_get_stage_times(gsht_plan *p, double *ms, int64_t *count, int nstages)
{
    if (!p || !ms || !count)
        return fail(GSHT_EINVAL, "plan/ms/count must not be NULL");
    for (int st = 0; st < ST_COUNT; ++st) {
        if (p->ev_pending[st]) {
            float t = 0;
            HIP_TRY(hipEventSynchronize(p->ev[2 * st + 1]));
            HIP_TRY(hipEventElapsedTime(&t, p->ev[2 * st], p->ev[2 * st + 1]));
            p->st_ms[st] += t;
            p->st_count[st] += 1;
            p->ev_pending[st] = 0;
        }
    }
    for (int st = 0; st < nstages && st < ST_COUNT; ++st) {
        ms[st] = p->st_ms[st];
        count[st] = p->st_count[st];
    }
    return ok();
}

int gsht_num_stages(void) { return ST_COUNT; }

const char *gsht_stage_name(int stage)
{
    if (stage < 0 || stage >= ST_COUNT)
        return "";
    return kStageNames[stage];
}

int gsht_legendre_rings(const void *alm, int lmax, int mmax, int spin, int ntheta,
                        gsht_precision prec, void *F, void *hip_stream)
{
    int rc = check_common(lmax, mmax, spin, 0, prec == GSHT_F64 ? 1e-10 : 1e-5, (int)prec);
    if (rc != GSHT_OK)
        return rc;
    if (ntheta < 2 || ntheta > 1 << 20)
        return fail(GSHT_EINVAL, "ntheta must be in [2, 2^20], got %d", ntheta);
    if (!alm || !F)
        return fail(GSHT_EINVAL, "alm/F must not be NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    gsht_plan *p = new gsht_plan();
    p->lmax = lmax;
    p->mmax = mmax;
    p->spin = spin;
    p->prec = (int)prec;
    p->ncomp = spin ? 2 : 1;
    p->nalm = (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
    p->ntheta = ntheta;
    p->nd = 2 * ntheta - 2;
    p->ncol = spin ? 2 * mmax + 1 : mmax + 1;
    p->npairs = (ntheta + 1) / 2;
    if ((rc = setup_legendre(p, s, false)) != GSHT_OK) { free_plan(p); return rc; }
    int rc2 = check_launch(launch_prep_alm(*p, alm, 1.0, false, s), "prep_alm");
    if (rc2 == GSHT_OK)
        rc2 = check_launch(launch_leg_synth(*p, F, false, s), "legendre_synth");
    if (rc2 == GSHT_OK)
        rc2 = check_launch(hipStreamSynchronize(s), "synchronize");
    free_plan(p);
    return rc2 == GSHT_OK ? ok() : rc2;
}

int gsht_analysis_minimal(const void *map, int lmax, int mmax, int spin, int nphi,
                          gsht_precision prec, void *alm, void *hip_stream)
{
    int rc = check_common(lmax, mmax, spin, 0, prec == GSHT_F64 ? 1e-10 : 1e-5, (int)prec);
    if (rc != GSHT_OK)
        return rc;
    if (nphi < 2 * mmax + 1 || nphi > 1 << 20)
        return fail(GSHT_EINVAL, "nphi must be in [2 mmax + 1, 2^20], got %d", nphi);
    if (!map || !alm)
        return fail(GSHT_EINVAL, "map/alm must not be NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    const int ntheta = lmax + 2, nd = 2 * lmax + 2, n2 = 2 * nd;
    const int ncol = spin ? 2 * mmax + 1 : mmax + 1;
    const size_t cs = prec == GSHT_F64 ? 16 : 8;
    // weights of the |sin| integral on the fine doubled grid (see analysis.hip)
    std::vector<double> u(n2);
    for (int i = 0; i < n2; ++i) {
        const long double t = 2.0L * (long double)M_PI * i / n2;
        long double acc = 4.0L;
        for (int n = 2; n <= 2 * lmax; n += 2)
            acc += 8.0L * cosl((long double)n * t) / (1.0L - (long double)n * n);
        u[i] = (double)(acc / n2);
    }
    void *P = nullptr, *D = nullptr, *Up = nullptr, *work = nullptr;
    double *du = nullptr;
    FFTPlan fphi, fnd, fn2;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        for (FFTPlan *f : {&fphi, &fnd, &fn2}) {
            if (f->info) rocfft_execution_info_destroy(f->info);
            if (f->plan) rocfft_plan_destroy(f->plan);
        }
        (void)hipFree(P);
        (void)hipFree(D);
        (void)hipFree(Up);
        (void)hipFree(work);
        (void)hipFree(du);
    };
#define AN_TRY(expr)                                                                              \
    do {                                                                                         \
        int rc_ = (expr);                                                                        \
        if (rc_ != GSHT_OK) {                                                                    \
            cleanup();                                                                           \
            return rc_;                                                                          \
        }                                                                                        \
    } while (0)
    auto halloc = [&](void **ptr, size_t bytes) {
        return hipMalloc(ptr, bytes) == hipSuccess ? GSHT_OK
                                                   : fail(GSHT_ENOMEM, "hipMalloc(%zu) failed", bytes);
    };
    AN_TRY(halloc(&P, (size_t)ntheta * nphi * cs));
    AN_TRY(halloc(&D, (size_t)ncol * nd * cs));
    AN_TRY(halloc(&Up, (size_t)ncol * n2 * cs));
    AN_TRY(halloc((void **)&du, sizeof(double) * n2));
    AN_TRY(make_fft(fphi, rocfft_transform_type_complex_forward, rocfft_placement_inplace, prec,
                    nphi, ntheta));
    AN_TRY(make_fft(fnd, rocfft_transform_type_complex_forward, rocfft_placement_inplace, prec, nd,
                    ncol));
    AN_TRY(make_fft(fn2, rocfft_transform_type_complex_inverse, rocfft_placement_inplace, prec, n2,
                    ncol));
    size_t wb = std::max(std::max(fphi.work_bytes, fnd.work_bytes), fn2.work_bytes);
    if (wb)
        AN_TRY(halloc(&work, wb));
    AN_TRY(check_launch(hipMemcpyAsync(du, u.data(), sizeof(double) * n2, hipMemcpyHostToDevice, s),
                        "weights"));
    // rings -> phi transforms -> doubled columns (phi quadrature weight 2 pi / nphi)
    AN_TRY(check_launch(launch_pack_rows(map, spin, (int64_t)ntheta * nphi, prec, P, s), "pack"));
    AN_TRY(run_fft(fphi, P, nullptr, work, wb, s));
    AN_TRY(check_launch(launch_gather_cols(P, ntheta, nphi, nd, mmax, spin, ncol,
                                           2.0 * M_PI / nphi, prec, D, s), "gather"));
    // theta weights in Fourier space, folded back onto the rings
    AN_TRY(run_fft(fnd, D, nullptr, work, wb, s));
    AN_TRY(check_launch(launch_pad_cols(D, nd, n2, lmax, ncol, 1.0 / nd, prec, Up, s), "pad"));
    AN_TRY(run_fft(fn2, Up, nullptr, work, wb, s));
    AN_TRY(check_launch(launch_weight_cols(Up, n2, ncol, du, prec, s), "weight"));
    AN_TRY(run_fft(fn2, Up, nullptr, work, wb, s));
    AN_TRY(check_launch(launch_trunc_cols(Up, nd, n2, lmax, ncol, 0.5 / nd, prec, D, s), "trunc"));
    AN_TRY(run_fft(fnd, D, nullptr, work, wb, s));
    // undoubling and adjoint Legendre step on the lmax + 2 rings
    gsht_plan *p = new gsht_plan();
    p->lmax = lmax;
    p->mmax = mmax;
    p->spin = spin;
    p->prec = (int)prec;
    p->ncomp = spin ? 2 : 1;
    p->nalm = (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
    p->ntheta = ntheta;
    p->nd = nd;
    p->ncol = ncol;
    p->npairs = (ntheta + 1) / 2;
    if ((rc = setup_legendre(p, s, false)) != GSHT_OK) {
        free_plan(p);
        cleanup();
        return rc;
    }
    int rc2 = check_launch(launch_leg_adjoint(*p, D, false, s), "legendre_adjoint");
    if (rc2 == GSHT_OK)
        rc2 = check_launch(launch_leg_finalize(*p, alm, 1.0, false, s), "finalize");
    if (rc2 == GSHT_OK)
        rc2 = check_launch(hipStreamSynchronize(s), "synchronize");
    free_plan(p);
    cleanup();
#undef AN_TRY
    return rc2 == GSHT_OK ? ok() : rc2;
}

int gsht_legendre_rings_adjoint(const void *F, int lmax, int mmax, int spin, int ntheta,
                                gsht_precision prec, void *alm, void *hip_stream)
{
    int rc = check_common(lmax, mmax, spin, 0, prec == GSHT_F64 ? 1e-10 : 1e-5, (int)prec);
    if (rc != GSHT_OK)
        return rc;
    if (ntheta < 2 || ntheta > 1 << 20)
        return fail(GSHT_EINVAL, "ntheta must be in [2, 2^20], got %d", ntheta);
    if (!alm || !F)
        return fail(GSHT_EINVAL, "alm/F must not be NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    gsht_plan *p = new gsht_plan();
    p->lmax = lmax;
    p->mmax = mmax;
    p->spin = spin;
    p->prec = (int)prec;
    p->ncomp = spin ? 2 : 1;
    p->nalm = (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
    p->ntheta = ntheta;
    p->nd = 2 * ntheta - 2;
    p->ncol = spin ? 2 * mmax + 1 : mmax + 1;
    p->npairs = (ntheta + 1) / 2;
    if ((rc = setup_legendre(p, s, false)) != GSHT_OK) { free_plan(p); return rc; }
    int rc2 = check_launch(launch_leg_adjoint(*p, F, false, s), "legendre_adjoint");
    if (rc2 == GSHT_OK)
        rc2 = check_launch(launch_leg_finalize(*p, alm, 1.0, false, s), "finalize");
    if (rc2 == GSHT_OK)
        rc2 = check_launch(hipStreamSynchronize(s), "synchronize");
    free_plan(p);
    return rc2 == GSHT_OK ? ok() : rc2;
}

int gsht_legendre_rings_adjoint_noalloc(const void *F, int lmax, int mmax, int spin, int ntheta,
                                        gsht_precision prec, void *alm, void *hip_stream)
{
    int rc = check_common(lmax, mmax, spin, 0, prec == GSHT_F64 ? 1e-10 : 1e-5, (int)prec);
    if (rc != GSHT_OK)
        return rc;
    if (ntheta < 2 || ntheta > 1 << 20)
        return fail(GSHT_EINVAL, "ntheta must be in [2, 2^20], got %d", ntheta);
    if (!alm || !F)
        return fail(GSHT_EINVAL, "alm/F must not be NULL");
    // the call's plan lives on the stack and points into the device scratch
    gsht_plan p;
    p.lmax = lmax;
    p.mmax = mmax;
    p.spin = spin;
    p.prec = (int)prec;
    p.ncomp = spin ? 2 : 1;
    p.nalm = (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
    p.ntheta = ntheta;
    p.nd = 2 * ntheta - 2;
    p.ncol = spin ? 2 * mmax + 1 : mmax + 1;
    p.npairs = (ntheta + 1) / 2;
    p.adj_nchunk = (p.npairs + 64 * p.adj_r - 1) / (64 * p.adj_r);
    p.syn_nchunk = (p.npairs + 64 * p.syn_r - 1) / (64 * p.syn_r);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_ab = up(sizeof(double2) * (size_t)p.nalm);
    const size_t b_norm = up(sizeof(double) * (size_t)p.nalm);
    const size_t b_acc = up(sizeof(double) * 2 * p.ncomp * (size_t)p.nalm);
    const size_t b_start = up(sizeof(StartInfo) * (size_t)(mmax + 1));
    const size_t b_live = up(sizeof(int32_t) * (size_t)(mmax + 1) * p.adj_nchunk);
    const size_t need = b_ab + b_norm + b_acc + b_start + b_live;
    if (need > kScratchBytes)
        return fail(GSHT_EINVAL, "lmax %d, mmax %d, spin %d, ntheta %d need %zu bytes of device "
                                 "scratch; the allocation-free entry point holds %zu",
                    lmax, mmax, spin, ntheta, need, kScratchBytes);
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    void *base = nullptr;
    if ((rc = scratch_address(dev, &base)) != GSHT_OK)
        return rc;
    char *q = (char *)base;
    p.leg.ab = (double2 *)q;
    q += b_ab;
    p.leg.norm = (double *)q;
    q += b_norm;
    p.acc = (double *)q;
    q += b_acc;
    p.leg.start = (StartInfo *)q;
    q += b_start;
    p.leg.lfirst_adj = (int32_t *)q;
    // start data: computed on the host, sent from a host copy kept until the next call
    g_scratch_start[dev] = make_start_info(lmax, mmax, spin);
    HIP_TRY(hipMemcpyAsync(p.leg.start, g_scratch_start[dev].data(),
                           sizeof(StartInfo) * (size_t)(mmax + 1), hipMemcpyHostToDevice, s));
    rc = check_launch(launch_leg_tables(p, s), "legendre tables");
    if (rc == GSHT_OK)
        rc = check_launch(launch_leg_live_adj(p, s), "live-chunk table");
    if (rc == GSHT_OK)
        rc = check_launch(launch_leg_adjoint(p, F, false, s), "legendre_adjoint");
    if (rc == GSHT_OK)
        rc = check_launch(launch_leg_finalize(p, alm, 1.0, false, s), "finalize");
    return rc == GSHT_OK ? ok() : rc;
}

}  // extern "C"

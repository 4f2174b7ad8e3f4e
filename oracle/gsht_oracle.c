/*
 * gsht_oracle.c -- TEST INFRASTRUCTURE ONLY.  Not part of the product path.
 *
 * A plain, slow, FP64 CPU reference for the general spin-weighted spherical
 * harmonic synthesis and its adjoint of Reinecke, Belkner & Carron (2023):
 *
 *   spin 0  (Sect. 2, eq. "forward"):   T_i = sum_{l<=lmax} sum_{|m|<=l} a_lm Y_lm(n_i)
 *   spin 0  (Sect. 2, eq. "adjoint"):   b_lm = sum_i T_i Y*_lm(n_i)
 *   spin s  (Sect. 2, eq. "forwardpol", chi = 0):
 *           P_i = - sum_{l,|m|<=l} (G_lm + i C_lm) sY_lm(n_i),   (Q, U) = (Re P, Im P)
 *   spin s adjoint (Sect. 2, the two-component adjoint and its gradient/curl split):
 *           S+_lm = sum_i (Q + iU)_i  sY*_lm(n_i),   S-_lm = sum_i (Q - iU)_i (-s)Y*_lm(n_i)
 *           G_lm = -(S+ + (-1)^s S-)/2,              C_lm = -(S+ - (-1)^s S-)/(2i)
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * load this library.  It shares no code, header or table with the GPU library.
 *
 * Conventions (the paper fixes none of these; they are the common public ones):
 *   - a_lm is stored for 0 <= m <= mmax, m <= l <= lmax only, m-major:
 *       idx(l, m) = m (2 lmax + 1 - m) / 2 + l, complex as (re, im) doubles.
 *     Each component (T, or G and C) is one such block; components follow
 *     each other.
 *   - Real-field convention: a_{l,-m} = (-1)^m conj(a_lm) for T, G and C, and
 *     only Re(a_l0) is used.
 *   - sY_lm is the Goldberg et al. (1967) spin-weighted harmonic
 *       sY_lm(th, ph) = (-1)^m sqrt[(l+m)!(l-m)!(2l+1) / (4 pi (l+s)!(l-s)!)]
 *                       sin^{2l}(th/2) sum_r C(l-s, r) C(l+s, r+s-m)
 *                       (-1)^{l-r-s} cot^{2r+s-m}(th/2) e^{i m ph},
 *     which is the Condon-Shortley spherical harmonic for s = 0.
 *
 * How sY_lm(theta) is evaluated for large l: at the first non-zero degree
 * l0 = max(|m|, |s|) the Goldberg sum has exactly one term, evaluated as
 * written (factorial ratio, half-angle powers).  Higher degrees follow the
 * standard three-term recurrence in l of the Wigner small-d function
 * d^l_{m,m'} (m' = -s), to which sY_lm is proportional with a factor
 * sqrt(2l+1) times an l-independent constant.  Because the start value can be
 * far below the double range (sin^m underflows long before l reaches the
 * turning point), every value is carried as (mantissa, binary exponent) and
 * rescaled by an exact power of two whenever it grows large.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

static int64_t alm_idx(int lmax, int l, int m)
{
    return (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2 + l;
}

static int64_t alm_count(int lmax, int mmax)
{
    return (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
}

/* ---- (mantissa, exponent) helpers: value = mant * 2^ex ------------------- */

typedef struct {
    double mant;
    long ex;
} xdouble;

static xdouble xnorm(double v, long ex)
{
    xdouble r;
    int e = 0;
    if (v == 0.0) {
        r.mant = 0.0;
        r.ex = 0;
        return r;
    }
    r.mant = frexp(v, &e);
    r.ex = ex + e;
    return r;
}

static xdouble xmul(xdouble a, xdouble b)
{
    return xnorm(a.mant * b.mant, a.ex + b.ex);
}

/* base^n for integer n >= 0, by binary exponentiation (0^0 = 1). */
static xdouble xpow(double base, int n)
{
    xdouble r = xnorm(1.0, 0);
    xdouble b = xnorm(base, 0);
    if (n == 0)
        return r;
    if (base == 0.0)
        return xnorm(0.0, 0);
    while (n > 0) {
        if (n & 1)
            r = xmul(r, b);
        b = xmul(b, b);
        n >>= 1;
    }
    return r;
}

/* ---- the start value at l0 = max(|m|, |s|) ---------------------------------- */

/* Unique summation index r of the Goldberg sum at l = l0 (see header). */
static int goldberg_r(int l0, int m, int s)
{
    int rlo = (m - s) > 0 ? (m - s) : 0;
    int rhi = (l0 - s) < (l0 + m) ? (l0 - s) : (l0 + m);
    return (rlo == rhi) ? rlo : -1;
}

/*
 * l-independent part of the single Goldberg term at l0:
 *   (-1)^m (-1)^{l0-r-s} sqrt[(2 l0 + 1)/(4 pi) * (l0+m)!(l0-m)!(l0-s)!(l0+s)!
 *                             / (r! (l0-s-r)! (r+s-m)! (l0+m-r)!)^2 ]
 * (the two binomials of the sum, squared and combined with the prefactor).
 * The factorial ratio is formed as prod_k k^{cnt[k]} so it never overflows.
 */
static xdouble start_prefactor(int l0, int m, int s)
{
    int r = goldberg_r(l0, m, s);
    int num[4] = {l0 + m, l0 - m, l0 - s, l0 + s};
    int den[4] = {r, l0 - s - r, r + s - m, l0 + m - r};
    int kmax = 2 * l0 + 1;
    int *cnt = (int *)calloc((size_t)kmax + 1, sizeof(int));
    xdouble acc = xnorm(1.0, 0);
    for (int i = 0; i < 4; ++i) {
        for (int k = 2; k <= num[i]; ++k)
            cnt[k] += 1;
        for (int k = 2; k <= den[i]; ++k)
            cnt[k] -= 2;
    }
    for (int k = 2; k <= kmax; ++k) {
        int c = cnt[k];
        while (c > 0) {
            acc = xmul(acc, xnorm((double)k, 0));
            --c;
        }
        while (c < 0) {
            acc = xmul(acc, xnorm(1.0 / (double)k, 0));
            ++c;
        }
    }
    free(cnt);
    acc = xmul(acc, xnorm((2.0 * l0 + 1.0) / (4.0 * M_PI), 0));
    /* square root of mant * 2^ex */
    if (acc.ex & 1) {
        acc.mant *= 2.0;
        acc.ex -= 1;
    }
    {
        xdouble root;
        root.mant = sqrt(acc.mant);
        root.ex = acc.ex / 2;
        root = xnorm(root.mant, root.ex);
        if (((m + (l0 - r - s)) & 1) != 0)
            root.mant = -root.mant;
        return root;
    }
}

/* ---- per-(m, s) recurrence tables ------------------------------------------ */

/*
 * With lam_l = sY_lm(theta, 0) (real), the Wigner-d recurrence (m' = -s) reads
 *   lam_{l+1} = (c1_l cos(theta) + c2_l) lam_l - c3_l lam_{l-1},   l >= l0,
 *   c1_l = sqrt((2l+3)/(2l+1)) (l+1)(2l+1) / sqrt(((l+1)^2 - m^2)((l+1)^2 - s^2))
 *   c2_l = c1_l m s / (l (l+1))          (0 when l = 0)
 *   c3_l = sqrt((2l+3)/(2l-1)) (l+1)(2l+1) / sqrt(((l+1)^2 - m^2)((l+1)^2 - s^2))
 *          * sqrt((l^2 - m^2)(l^2 - s^2)) / (l (2l+1))     (0 when l = l0)
 */
typedef struct {
    int l0;
    int a_sin, b_cos; /* half-angle exponents of the start term */
    xdouble pref;
    double *c1, *c2, *c3; /* indexed by l, valid for l0 <= l < lmax */
} rec_table;

static int rec_table_init(rec_table *t, int lmax, int m, int s)
{
    int am = m < 0 ? -m : m, as = s < 0 ? -s : s;
    t->l0 = am > as ? am : as;
    t->c1 = t->c2 = t->c3 = NULL;
    if (t->l0 > lmax)
        return ORACLE_OK;
    {
        int r = goldberg_r(t->l0, m, s);
        if (r < 0)
            return ORACLE_EINVAL;
        t->b_cos = 2 * r + s - m;
        t->a_sin = 2 * t->l0 - t->b_cos;
        t->pref = start_prefactor(t->l0, m, s);
    }
    t->c1 = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
    t->c2 = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
    t->c3 = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
    if (!t->c1 || !t->c2 || !t->c3)
        return ORACLE_ENOMEM;
    for (int l = t->l0; l < lmax; ++l) {
        double L = (double)l;
        double q = ((L + 1) * (L + 1) - (double)m * m) * ((L + 1) * (L + 1) - (double)s * s);
        double A = (L + 1) * (2 * L + 1) / sqrt(q);
        t->c1[l] = sqrt((2 * L + 3) / (2 * L + 1)) * A;
        t->c2[l] = (l == 0) ? 0.0 : t->c1[l] * (double)m * (double)s / (L * (L + 1));
        if (l == t->l0 || l == 0)
            t->c3[l] = 0.0;
        else
            t->c3[l] = sqrt((2 * L + 3) / (2 * L - 1)) * A *
                       sqrt((L * L - (double)m * m) * (L * L - (double)s * s)) / (L * (2 * L + 1));
    }
    return ORACLE_OK;
}

static void rec_table_free(rec_table *t)
{
    free(t->c1);
    free(t->c2);
    free(t->c3);
}

/*
 * Walk l = l0..lmax at one theta and call back with the true value of
 * sY_lm(theta, 0).  The running pair (v0, v1) shares the exponent ex; the true
 * value is ldexp(v1, ex), which is exact or underflows to the correctly
 * rounded tiny value.
 */
#define WALK_BEGIN(T, LMAX, THETA)                                                   \
    {                                                                                \
        const rec_table *wt_ = (T);                                                  \
        double x_ = cos(THETA);                                                      \
        xdouble st_ = xmul(wt_->pref, xmul(xpow(sin(0.5 * (THETA)), wt_->a_sin),     \
                                           xpow(cos(0.5 * (THETA)), wt_->b_cos)));   \
        double v0_ = 0.0, v1_ = st_.mant;                                            \
        long ex_ = st_.ex;                                                           \
        for (int l = wt_->l0; l <= (LMAX); ++l) {                                    \
            double lam = (ex_ < -2200) ? 0.0 : ldexp(v1_, (int)ex_);

#define WALK_END(LMAX)                                                               \
            if (l < (LMAX)) {                                                        \
                double v2_ = (wt_->c1[l] * x_ + wt_->c2[l]) * v1_ - wt_->c3[l] * v0_;\
                v0_ = v1_;                                                           \
                v1_ = v2_;                                                           \
                if (fabs(v1_) > 0x1p+300) {                                          \
                    v0_ = ldexp(v0_, -600);                                          \
                    v1_ = ldexp(v1_, -600);                                          \
                    ex_ += 600;                                                      \
                }                                                                    \
            }                                                                        \
        }                                                                            \
    }

/* sY_lm(theta, 0) for l = 0..lmax (zero below l0).  Any integer m and s. */
int gsht_oracle_slambda(int lmax, int m, int s, double theta, double *out)
{
    rec_table t;
    int rc;
    if (lmax < 0 || !out)
        return ORACLE_EINVAL;
    memset(out, 0, sizeof(double) * (size_t)(lmax + 1));
    rc = rec_table_init(&t, lmax, m, s);
    if (rc != ORACLE_OK || t.l0 > lmax) {
        rec_table_free(&t);
        return rc;
    }
    WALK_BEGIN(&t, lmax, theta)
    out[l] = lam;
    WALK_END(lmax)
    rec_table_free(&t);
    return ORACLE_OK;
}

/* Full complex coefficient c_lm for -l <= m <= l from the stored m >= 0 block. */
static void full_coef(const double *blk, int lmax, int l, int m, double *re, double *im)
{
    int am = m < 0 ? -m : m;
    const double *c = blk + 2 * alm_idx(lmax, l, am);
    double cr = c[0], ci = (am == 0) ? 0.0 : c[1];
    if (m < 0) { /* (-1)^m conj(a_l|m|) */
        double sg = (am & 1) ? -1.0 : 1.0;
        cr = sg * cr;
        ci = -sg * ci;
    }
    *re = cr;
    *im = ci;
}

static int nthreads_or_default(int n)
{
#ifdef _OPENMP
    return n > 0 ? n : omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/*
 * Direct-sum synthesis.
 * alm: [ncomp][nalm] complex (re, im), ncomp = 1 (spin 0) or 2 (G, C).
 * map: [ncomp][npts] real: T, or (Q, U).
 * Parallel over m; each thread owns a private map, summed in thread order.
 */
int gsht_oracle_synth(const double *alm, int lmax, int mmax, int spin, int64_t npts,
                      const double *theta, const double *phi, double *map, int nthreads)
{
    int nt = nthreads_or_default(nthreads);
    int64_t nalm;
    double *priv;
    int status = ORACLE_OK;
    if (lmax < 0 || mmax < 0 || mmax > lmax || spin < 0 || spin > lmax || npts < 0)
        return ORACLE_EINVAL;
    nalm = alm_count(lmax, mmax);
    priv = (double *)calloc((size_t)nt * 2 * (size_t)(npts > 0 ? npts : 1), sizeof(double));
    if (!priv)
        return ORACLE_ENOMEM;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = priv + (size_t)tid * 2 * (size_t)npts; /* complex per point */
#pragma omp for schedule(dynamic, 1)
        for (int mm = -mmax; mm <= mmax; ++mm) {
            rec_table t;
            double *cr = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
            double *ci = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
            if (rec_table_init(&t, lmax, mm, spin) != ORACLE_OK || !cr || !ci) {
#pragma omp atomic write
                status = ORACLE_ENOMEM;
            } else if (t.l0 <= lmax) {
                /* c_lm = a_lm (spin 0) or -(G_lm + i C_lm) (spin > 0) */
                for (int l = t.l0; l <= lmax; ++l) {
                    if (spin == 0) {
                        full_coef(alm, lmax, l, mm, &cr[l], &ci[l]);
                    } else {
                        double gr, gi, xr, xi;
                        full_coef(alm, lmax, l, mm, &gr, &gi);
                        full_coef(alm + 2 * nalm, lmax, l, mm, &xr, &xi);
                        cr[l] = -(gr - xi);
                        ci[l] = -(gi + xr);
                    }
                }
                for (int64_t i = 0; i < npts; ++i) {
                    double sr = 0.0, si = 0.0;
                    WALK_BEGIN(&t, lmax, theta[i])
                    sr += cr[l] * lam;
                    si += ci[l] * lam;
                    WALK_END(lmax)
                    {
                        double c = cos(mm * phi[i]), s = sin(mm * phi[i]);
                        acc[2 * i] += sr * c - si * s;
                        acc[2 * i + 1] += sr * s + si * c;
                    }
                }
            }
            rec_table_free(&t);
            free(cr);
            free(ci);
        }
    }
    for (int64_t i = 0; i < npts; ++i) {
        double re = 0.0, im = 0.0;
        for (int t = 0; t < nt; ++t) {
            re += priv[(size_t)t * 2 * npts + 2 * i];
            im += priv[(size_t)t * 2 * npts + 2 * i + 1];
        }
        map[i] = re; /* spin 0: the imaginary part is zero by symmetry */
        if (spin > 0)
            map[npts + i] = im;
    }
    free(priv);
    return status;
}

/*
 * Direct-sum adjoint for one m >= 0: the coefficients (l, m), l = m..lmax, of every
 * component, written into alm ([ncomp][nalm] complex).  Returns ORACLE_ENOMEM on
 * allocation failure.
 */
static int adjoint_one_m(const double *map, int lmax, int spin, int64_t npts, const double *theta,
                         const double *phi, int64_t nalm, int m, double *alm)
{
    rec_table tp = {0}, tm = {0};
    double *sp = (double *)calloc(2 * (size_t)(lmax + 1), sizeof(double));
    double *sm = (double *)calloc(2 * (size_t)(lmax + 1), sizeof(double));
    int ok = sp && sm && rec_table_init(&tp, lmax, m, spin) == ORACLE_OK;
    if (ok && spin > 0)
        ok = rec_table_init(&tm, lmax, m, -spin) == ORACLE_OK;
    if (ok) {
        for (int64_t i = 0; i < npts; ++i) {
            double c = cos(m * phi[i]), s = sin(m * phi[i]);
            /* +s part: (Q + iU) e^{-i m phi} sY_lm ; spin 0: T e^{-i m phi} Y_lm */
            double q = map[i], u = (spin > 0) ? map[npts + i] : 0.0;
            double pr = q * c + u * s, pi = u * c - q * s;
            if (tp.l0 <= lmax) {
                WALK_BEGIN(&tp, lmax, theta[i])
                sp[2 * l] += pr * lam;
                sp[2 * l + 1] += pi * lam;
                WALK_END(lmax)
            }
            if (spin > 0 && tm.l0 <= lmax) {
                /* -s part: (Q - iU) e^{-i m phi} (-s)Y_lm */
                double nr = q * c - u * s, ni = -u * c - q * s;
                WALK_BEGIN(&tm, lmax, theta[i])
                sm[2 * l] += nr * lam;
                sm[2 * l + 1] += ni * lam;
                WALK_END(lmax)
            }
        }
        for (int l = m; l <= lmax; ++l) {
            double *g = alm + 2 * alm_idx(lmax, l, m);
            if (l < spin)
                continue;
            if (spin == 0) {
                g[0] = sp[2 * l];
                g[1] = (m == 0) ? 0.0 : sp[2 * l + 1];
            } else {
                double sg = (spin & 1) ? -1.0 : 1.0;
                double ar = sp[2 * l] + sg * sm[2 * l], ai = sp[2 * l + 1] + sg * sm[2 * l + 1];
                double br = sp[2 * l] - sg * sm[2 * l], bi = sp[2 * l + 1] - sg * sm[2 * l + 1];
                double *cc = g + 2 * nalm;
                g[0] = -0.5 * ar;                  /* G = -(S+ + (-1)^s S-)/2   */
                g[1] = (m == 0) ? 0.0 : -0.5 * ai;
                cc[0] = -0.5 * bi;                 /* C = -(S+ - (-1)^s S-)/(2i) */
                cc[1] = (m == 0) ? 0.0 : 0.5 * br;
            }
        }
    }
    rec_table_free(&tp);
    rec_table_free(&tm);
    free(sp);
    free(sm);
    return ok ? ORACLE_OK : ORACLE_ENOMEM;
}

/*
 * Direct-sum adjoint.  map: [ncomp][npts] real; alm out: [ncomp][nalm] complex.
 * Parallel over m >= 0; each m is owned by one thread.
 */
int gsht_oracle_adjoint(const double *map, int lmax, int mmax, int spin, int64_t npts,
                        const double *theta, const double *phi, double *alm, int nthreads)
{
    int nt = nthreads_or_default(nthreads);
    int64_t nalm;
    int status = ORACLE_OK;
    if (lmax < 0 || mmax < 0 || mmax > lmax || spin < 0 || spin > lmax || npts < 0)
        return ORACLE_EINVAL;
    nalm = alm_count(lmax, mmax);
    memset(alm, 0, sizeof(double) * 2 * (size_t)nalm * (spin > 0 ? 2 : 1));
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int m = 0; m <= mmax; ++m) {
        if (adjoint_one_m(map, lmax, spin, npts, theta, phi, nalm, m, alm) != ORACLE_OK) {
#pragma omp atomic write
            status = ORACLE_ENOMEM;
        }
    }
    return status;
}

/*
 * The same adjoint for the listed m values only (each in [0, mmax], no repeats):
 * their coefficients as gsht_oracle_adjoint gives them, every other entry of alm
 * zero.  Lets a test check sampled outputs of a large adjoint one column at a time.
 */
int gsht_oracle_adjoint_cols(const double *map, int lmax, int mmax, int spin, int64_t npts,
                             const double *theta, const double *phi, const int32_t *mlist,
                             int nm, double *alm, int nthreads)
{
    int nt = nthreads_or_default(nthreads);
    int64_t nalm;
    int status = ORACLE_OK;
    if (lmax < 0 || mmax < 0 || mmax > lmax || spin < 0 || spin > lmax || npts < 0 || nm < 0)
        return ORACLE_EINVAL;
    for (int k = 0; k < nm; ++k) {
        if (mlist[k] < 0 || mlist[k] > mmax)
            return ORACLE_EINVAL;
        for (int j = 0; j < k; ++j)
            if (mlist[j] == mlist[k])
                return ORACLE_EINVAL;
    }
    nalm = alm_count(lmax, mmax);
    memset(alm, 0, sizeof(double) * 2 * (size_t)nalm * (spin > 0 ? 2 : 1));
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int k = 0; k < nm; ++k) {
        if (adjoint_one_m(map, lmax, spin, npts, theta, phi, nalm, mlist[k], alm) != ORACLE_OK) {
#pragma omp atomic write
            status = ORACLE_ENOMEM;
        }
    }
    return status;
}

/*
 * Ring synthesis in (theta, m) space: F_m(theta_j) = sum_l c_lm sY_lm(theta_j, 0)
 * for -mmax <= m <= mmax, with c_lm the full coefficient used by
 * gsht_oracle_synth (a_lm, or -(G_lm + i C_lm)).  Then the map on ring j is
 * sum_m F_m(theta_j) e^{i m phi}.   F: [2 mmax + 1][nring] complex, row m + mmax.
 */
int gsht_oracle_ring_synth(const double *alm, int lmax, int mmax, int spin, int nring,
                           const double *theta, double *F, int nthreads)
{
    int nt = nthreads_or_default(nthreads);
    int64_t nalm;
    int status = ORACLE_OK;
    if (lmax < 0 || mmax < 0 || mmax > lmax || spin < 0 || spin > lmax || nring < 0)
        return ORACLE_EINVAL;
    nalm = alm_count(lmax, mmax);
    memset(F, 0, sizeof(double) * 2 * (size_t)(2 * mmax + 1) * (size_t)nring);
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int mm = -mmax; mm <= mmax; ++mm) {
        rec_table t;
        if (rec_table_init(&t, lmax, mm, spin) != ORACLE_OK) {
#pragma omp atomic write
            status = ORACLE_ENOMEM;
        } else if (t.l0 <= lmax) {
            double *row = F + 2 * (size_t)(mm + mmax) * (size_t)nring;
            for (int j = 0; j < nring; ++j) {
                double sr = 0.0, si = 0.0;
                WALK_BEGIN(&t, lmax, theta[j])
                double cr, ci;
                if (spin == 0) {
                    full_coef(alm, lmax, l, mm, &cr, &ci);
                } else {
                    double gr, gi, xr, xi;
                    full_coef(alm, lmax, l, mm, &gr, &gi);
                    full_coef(alm + 2 * nalm, lmax, l, mm, &xr, &xi);
                    cr = -(gr - xi);
                    ci = -(gi + xr);
                }
                sr += cr * lam;
                si += ci * lam;
                WALK_END(lmax)
                row[2 * j] = sr;
                row[2 * j + 1] = si;
            }
        }
        rec_table_free(&t);
    }
    return status;
}

/*
 * Ring adjoint in (theta, m) space.  Input H_m(theta_j) = sum_k P(theta_j, phi_k)
 * e^{-i m phi_k} for -mmax <= m <= mmax ([2 mmax + 1][nring] complex; for spin 0 only
 * rows m >= 0 are read).  Output as gsht_oracle_adjoint would give for points on
 * those rings:  spin 0:  b_lm = sum_j Y_lm(theta_j, 0) H_m(theta_j);
 * spin s:  S+_lm = sum_j sY_lm H_m,  S-_lm = sum_j (-s)Y_lm conj(H_{-m}),
 * then the gradient/curl combination.
 */
int gsht_oracle_ring_adjoint(const double *H, int lmax, int mmax, int spin, int nring,
                             const double *theta, double *alm, int nthreads)
{
    int nt = nthreads_or_default(nthreads);
    int64_t nalm;
    int status = ORACLE_OK;
    if (lmax < 0 || mmax < 0 || mmax > lmax || spin < 0 || spin > lmax || nring < 0)
        return ORACLE_EINVAL;
    nalm = alm_count(lmax, mmax);
    memset(alm, 0, sizeof(double) * 2 * (size_t)nalm * (spin > 0 ? 2 : 1));
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int m = 0; m <= mmax; ++m) {
        rec_table tp = {0}, tm = {0};
        double *sp = (double *)calloc(2 * (size_t)(lmax + 1), sizeof(double));
        double *sm = (double *)calloc(2 * (size_t)(lmax + 1), sizeof(double));
        const double *hp = H + 2 * (size_t)(m + mmax) * (size_t)nring;
        const double *hm = H + 2 * (size_t)(-m + mmax) * (size_t)nring;
        int ok = sp && sm && rec_table_init(&tp, lmax, m, spin) == ORACLE_OK;
        if (ok && spin > 0)
            ok = rec_table_init(&tm, lmax, m, -spin) == ORACLE_OK;
        if (!ok) {
#pragma omp atomic write
            status = ORACLE_ENOMEM;
        } else {
            for (int j = 0; j < nring; ++j) {
                if (tp.l0 <= lmax) {
                    WALK_BEGIN(&tp, lmax, theta[j])
                    sp[2 * l] += hp[2 * j] * lam;
                    sp[2 * l + 1] += hp[2 * j + 1] * lam;
                    WALK_END(lmax)
                }
                if (spin > 0 && tm.l0 <= lmax) {
                    WALK_BEGIN(&tm, lmax, theta[j])
                    sm[2 * l] += hm[2 * j] * lam;
                    sm[2 * l + 1] -= hm[2 * j + 1] * lam;
                    WALK_END(lmax)
                }
            }
            for (int l = m; l <= lmax; ++l) {
                double *g = alm + 2 * alm_idx(lmax, l, m);
                if (l < spin)
                    continue;
                if (spin == 0) {
                    g[0] = sp[2 * l];
                    g[1] = (m == 0) ? 0.0 : sp[2 * l + 1];
                } else {
                    double sg = (spin & 1) ? -1.0 : 1.0;
                    double ar = sp[2 * l] + sg * sm[2 * l], ai = sp[2 * l + 1] + sg * sm[2 * l + 1];
                    double br = sp[2 * l] - sg * sm[2 * l], bi = sp[2 * l + 1] - sg * sm[2 * l + 1];
                    double *cc = g + 2 * nalm;
                    g[0] = -0.5 * ar;
                    g[1] = (m == 0) ? 0.0 : -0.5 * ai;
                    cc[0] = -0.5 * bi;
                    cc[1] = (m == 0) ? 0.0 : 0.5 * br;
                }
            }
        }
        rec_table_free(&tp);
        rec_table_free(&tm);
        free(sp);
        free(sm);
    }
    return status;
}

/*
 * ---- Plain NUFFT steps of the FFT-based general SHT (Sect. 3) ----------------
 *
 * The grid is the whole periodic N1 x N2 torus (theta in [0, 2 pi) after the
 * doubling, phi in [0, 2 pi)), complex, row-major g[a][b], cell sizes
 * h1 = 2 pi / N1, h2 = 2 pi / N2.  The kernel in cell units is
 *     psi(t) = exp(beta (sqrt(1 - (2t/w)^2) - 1))   for |t| <= w/2, else 0,
 * the "exponential of semicircle" kernel with support w cells.  A point at
 * (u, v) = (theta N1 / 2 pi, phi N2 / 2 pi) touches the w x w cells
 * a = a0 .. a0 + w - 1, b = b0 .. b0 + w - 1, a0 = ceil(u - w/2),
 * b0 = ceil(v - w/2), taken modulo N1 and N2.
 */
static double es_psi(double t, int w, double beta)
{
    double z = 2.0 * t / w;
    if (z * z > 1.0)
        return 0.0;
    return exp(beta * (sqrt(1.0 - z * z) - 1.0));
}

static int64_t wrap_index(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

static int nufft_args_ok(int n1, int n2, int w, int64_t npts)
{
    return n1 >= w && n2 >= w && w >= 1 && w <= 32 && npts >= 0;
}

/* Type-2 step (uniform grid -> points): out_i = sum_{a,b} g[a][b] psi(u_i - a) psi(v_i - b). */
int gsht_oracle_nufft_interp(const double *g, int n1, int n2, int w, double beta, int64_t npts,
                             const double *theta, const double *phi, double *out, int nthreads)
{
    int nt = nthreads_or_default(nthreads);
    const double c1 = (double)n1 / (2.0 * M_PI), c2 = (double)n2 / (2.0 * M_PI);
    if (!nufft_args_ok(n1, n2, w, npts))
        return ORACLE_EINVAL;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
        double u = theta[i] * c1, v = phi[i] * c2, pb[32];
        int64_t a0 = (int64_t)ceil(u - 0.5 * w), b0 = (int64_t)ceil(v - 0.5 * w);
        double sr = 0.0, si = 0.0;
        for (int db = 0; db < w; ++db)
            pb[db] = es_psi(v - (double)(b0 + db), w, beta);
        for (int da = 0; da < w; ++da) {
            double pa = es_psi(u - (double)(a0 + da), w, beta);
            const double *row = g + 2 * (size_t)wrap_index(a0 + da, n1) * (size_t)n2;
            for (int db = 0; db < w; ++db) {
                double k = pa * pb[db];
                const double *c = row + 2 * wrap_index(b0 + db, n2);
                sr += c[0] * k;
                si += c[1] * k;
            }
        }
        out[2 * i] = sr;
        out[2 * i + 1] = si;
    }
    return ORACLE_OK;
}

/* Type-1 step (points -> uniform grid), the exact transpose of the type-2 step:
 * g[a][b] += y_i psi(u_i - a) psi(v_i - b).  g is accumulated, not cleared.  One
 * thread: points are added in input order. */
int gsht_oracle_nufft_spread(const double *y, int n1, int n2, int w, double beta, int64_t npts,
                             const double *theta, const double *phi, double *g)
{
    const double c1 = (double)n1 / (2.0 * M_PI), c2 = (double)n2 / (2.0 * M_PI);
    if (!nufft_args_ok(n1, n2, w, npts))
        return ORACLE_EINVAL;
    for (int64_t i = 0; i < npts; ++i) {
        double u = theta[i] * c1, v = phi[i] * c2, pb[32];
        int64_t a0 = (int64_t)ceil(u - 0.5 * w), b0 = (int64_t)ceil(v - 0.5 * w);
        for (int db = 0; db < w; ++db)
            pb[db] = es_psi(v - (double)(b0 + db), w, beta);
        for (int da = 0; da < w; ++da) {
            double pa = es_psi(u - (double)(a0 + da), w, beta);
            double *row = g + 2 * (size_t)wrap_index(a0 + da, n1) * (size_t)n2;
            for (int db = 0; db < w; ++db) {
                double k = pa * pb[db];
                double *c = row + 2 * wrap_index(b0 + db, n2);
                c[0] += y[2 * i] * k;
                c[1] += y[2 * i + 1] * k;
            }
        }
    }
    return ORACLE_OK;
}

/*
 * Derivatives of the direct-sum synthesis with respect to the point coordinates:
 *   d/dphi:   each term c_lm sY_lm(theta) e^{i m phi} gains the factor i m;
 *   d/dtheta: the spin-weighted ladder relation
 *     d/dtheta sY_lm = -(1/2) [ sqrt((l-s)(l+s+1)) (s+1)Y_lm - sqrt((l+s)(l-s+1)) (s-1)Y_lm ],
 *   evaluated with the recurrences of spins s + 1 and s - 1.
 * dth, dph: [ncomp][npts] real (derivatives of T, or of Q and U).  Serial over
 * points is not needed: parallel over m with private accumulators, as the synthesis.
 */
int gsht_oracle_synth_deriv(const double *alm, int lmax, int mmax, int spin, int64_t npts,
                            const double *theta, const double *phi, double *dth, double *dph,
                            int nthreads)
{
    int nt = nthreads_or_default(nthreads);
    int64_t nalm;
    double *priv;
    int status = ORACLE_OK;
    if (lmax < 0 || mmax < 0 || mmax > lmax || spin < 0 || spin > lmax || npts < 0)
        return ORACLE_EINVAL;
    nalm = alm_count(lmax, mmax);
    priv = (double *)calloc((size_t)nt * 4 * (size_t)(npts > 0 ? npts : 1), sizeof(double));
    if (!priv)
        return ORACLE_ENOMEM;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = priv + (size_t)tid * 4 * (size_t)npts; /* (dtheta, dphi) complex */
#pragma omp for schedule(dynamic, 1)
        for (int mm = -mmax; mm <= mmax; ++mm) {
            rec_table t0 = {0}, tp = {0}, tm = {0};
            double *cr = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
            double *ci = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
            int ok = cr && ci && rec_table_init(&t0, lmax, mm, spin) == ORACLE_OK &&
                     rec_table_init(&tp, lmax, mm, spin + 1) == ORACLE_OK &&
                     rec_table_init(&tm, lmax, mm, spin - 1) == ORACLE_OK;
            if (!ok) {
#pragma omp atomic write
                status = ORACLE_ENOMEM;
            } else if (t0.l0 <= lmax) {
                for (int l = t0.l0; l <= lmax; ++l) {
                    if (spin == 0) {
                        full_coef(alm, lmax, l, mm, &cr[l], &ci[l]);
                    } else {
                        double gr, gi, xr, xi;
                        full_coef(alm, lmax, l, mm, &gr, &gi);
                        full_coef(alm + 2 * nalm, lmax, l, mm, &xr, &xi);
                        cr[l] = -(gr - xi);
                        ci[l] = -(gi + xr);
                    }
                }
                for (int64_t i = 0; i < npts; ++i) {
                    double sr = 0.0, si = 0.0, ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
                    WALK_BEGIN(&t0, lmax, theta[i])
                    if (l >= t0.l0) {
                        sr += cr[l] * lam;
                        si += ci[l] * lam;
                    }
                    WALK_END(lmax)
                    if (tp.l0 <= lmax) {
                        WALK_BEGIN(&tp, lmax, theta[i])
                        if (l >= t0.l0) {
                            double f = sqrt((double)(l - spin) * (double)(l + spin + 1)) * lam;
                            ar += cr[l] * f;
                            ai += ci[l] * f;
                        }
                        WALK_END(lmax)
                    }
                    if (tm.l0 <= lmax) {
                        WALK_BEGIN(&tm, lmax, theta[i])
                        if (l >= t0.l0) {
                            double f = sqrt((double)(l + spin) * (double)(l - spin + 1)) * lam;
                            br += cr[l] * f;
                            bi += ci[l] * f;
                        }
                        WALK_END(lmax)
                    }
                    {
                        double c = cos(mm * phi[i]), s = sin(mm * phi[i]);
                        double tr = -0.5 * (ar - br), ti = -0.5 * (ai - bi);
                        /* d/dphi: i m (sr + i si) */
                        double pr = -mm * si, pi = mm * sr;
                        acc[4 * i] += tr * c - ti * s;
                        acc[4 * i + 1] += tr * s + ti * c;
                        acc[4 * i + 2] += pr * c - pi * s;
                        acc[4 * i + 3] += pr * s + pi * c;
                    }
                }
            }
            rec_table_free(&t0);
            rec_table_free(&tp);
            rec_table_free(&tm);
            free(cr);
            free(ci);
        }
    }
    for (int64_t i = 0; i < npts; ++i) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int t = 0; t < nt; ++t)
            for (int k = 0; k < 4; ++k)
                v[k] += priv[(size_t)t * 4 * npts + 4 * i + k];
        dth[i] = v[0];
        dph[i] = v[2];
        if (spin > 0) {
            dth[npts + i] = v[1];
            dph[npts + i] = v[3];
        }
    }
    free(priv);
    return status;
}

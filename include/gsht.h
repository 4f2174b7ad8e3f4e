/*
 * gsht.h -- general spin-weighted spherical harmonic synthesis and its adjoint
 * on arbitrary points, for AMD Instinct MI355X (gfx950).
 *
 * The operations are those of Reinecke, Belkner & Carron (2023), "Improved CMB
 * (de-)lensing using general spherical harmonic transforms":
 *
 *   synthesis (Sect. 2, eq. "forward" for spin 0, eq. "forwardpol" with chi = 0
 *   for spin s > 0):
 *       spin 0:  T_i = sum_{l <= lmax} sum_{|m| <= min(l, mmax)} a_lm  Y_lm(theta_i, phi_i)
 *       spin s:  Q_i + i U_i = - sum_{l, |m|} (G_lm + i C_lm) sY_lm(theta_i, phi_i)
 *   adjoint (Sect. 2, eq. "adjoint" and the gradient/curl split that follows
 *   eq. "forwardpol"):
 *       spin 0:  b_lm = sum_i T_i Y*_lm(theta_i, phi_i)
 *       spin s:  S+_lm = sum_i (Q + iU)_i sY*_lm,  S-_lm = sum_i (Q - iU)_i (-s)Y*_lm,
 *                G_lm = -(S+ + (-1)^s S-)/2,        C_lm = -(S+ - (-1)^s S-)/(2i)
 *
 * computed as in Sect. 3: ring-by-ring Legendre synthesis onto an equidistant
 * (Clenshaw-Curtis) ring grid with ntheta >= lmax + 2 rings including both poles,
 * doubling of the theta range to a 2-D torus with the (-1)^(s+m) mirror sign, a
 * 2-D FFT with correction by the kernel's Fourier transform, and a type-2 NUFFT
 * (interpolation with an exponential-of-semicircle kernel) onto the points.  The
 * adjoint runs the type-1 NUFFT (spreading), the FFT back, undoubling and the
 * adjoint Legendre step.  The NUFFT is the only approximate step; its relative
 * L2 error is controlled by epsilon (Sect. 3; accuracy metric of Sect. 4).
 *
 * Common conventions of every entry point
 *   - All array pointers are DEVICE pointers (hipMalloc'd or equivalent) unless a
 *     parameter says otherwise.  The caller owns every buffer it passes; the
 *     library never frees or retains caller memory beyond the call, except that
 *     a plan keeps its own sorted copy of the point coordinates.
 *   - a_lm layout: complex, m-major triangular, one block per component:
 *       idx(l, m) = m (2 lmax + 1 - m) / 2 + l,  0 <= m <= mmax,  m <= l <= lmax,
 *       nalm = (mmax + 1)(lmax + 1) - mmax (mmax + 1) / 2,  array [ncomp][nalm].
 *     ncomp = 1 (T) for spin 0 and 2 (G, C) for spin > 0.  Real-field convention
 *     a_{l,-m} = (-1)^m conj(a_lm).  Imag(a_l0) and entries with l < spin are
 *     ignored by the synthesis and returned as exactly 0 by the adjoint.
 *   - Maps: real, [ncomp][npts]: T for spin 0, (Q, U) for spin > 0.
 *   - theta, phi: FP64 in every precision.  theta must lie in [0, pi]; phi may be
 *     any value with |phi| <= 2^20 (it is wrapped modulo 2 pi on the grid; the
 *     kernel offsets carry an absolute error of about |phi| 2^-52, so accuracy
 *     is as stated for |phi| of order 2 pi).  Other values give GSHT_EINVAL.
 *   - Precision GSHT_F64: a_lm complex128, maps float64, FFT/NUFFT in FP64,
 *     1e-13 <= epsilon <= 0.1.  GSHT_F32: a_lm complex64, maps float32, FFT and
 *     NUFFT in FP32 with FP64 point-to-grid offsets, 1e-5 <= epsilon <= 0.1.  The
 *     Legendre recurrence is FP64 in both.
 *   - Streams: hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it and the call returns without waiting, except where noted.
 *     Inputs must stay unchanged until the stream has reached the call.
 *   - Errors: every function returns a gsht_status; it never aborts or throws.
 *     Invalid arguments are rejected before any device work.  gsht_last_error()
 *     returns a thread-local message describing the last non-OK status.
 */
#ifndef GSHT_H
#define GSHT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSHT_OK = 0,
    GSHT_EINVAL = -1,       /* invalid argument (sizes, ranges, NULL, theta outside [0, pi], NaN) */
    GSHT_ENOMEM = -2,       /* device or host allocation failed, or above GSHT_MAX_WORKSPACE_BYTES */
    GSHT_EHIP = -3,         /* a HIP or rocFFT call failed; see gsht_last_error() */
    GSHT_EUNSUPPORTED = -4  /* valid request this build does not support (e.g. npts >= 2^31) */
} gsht_status;

typedef enum { GSHT_F64 = 0, GSHT_F32 = 1 } gsht_precision;

/* Opaque plan: geometry (sorted points), grid sizes, FFT plans and workspace. */
typedef struct gsht_plan gsht_plan;

/*
 * One-shot synthesis (Sect. 2, eq. "forward" / "forwardpol"; steps of Sect. 3).
 *   alm   [ncomp][nalm] complex (complex128 for F64, complex64 for F32), read only.
 *   map   [ncomp][npts] real (float64 / float32), overwritten.
 * Builds a plan (bin sort of the points, FFT plans, workspace), runs it and
 * frees it; the plan construction synchronises hip_stream once to validate
 * the coordinates.  Use the plan API below to reuse a geometry.
 */
int gsht_synth_general(const void *alm, int lmax, int mmax, int spin,
                       const double *theta, const double *phi, int64_t npts,
                       double epsilon, gsht_precision prec, void *map, void *hip_stream);

/*
 * One-shot adjoint synthesis (Sect. 2, eq. "adjoint" and the gradient/curl split;
 * the reversed steps of Sect. 3).
 *   map   [ncomp][npts] real, read only.
 *   alm   [ncomp][nalm] complex, overwritten (not accumulated).
 * Same plan handling as gsht_synth_general.
 */
int gsht_adjoint_synth_general(const void *map, int lmax, int mmax, int spin,
                               const double *theta, const double *phi, int64_t npts,
                               double epsilon, gsht_precision prec, void *alm,
                               void *hip_stream);

/*
 * Map analysis on the minimal equiangular grid (Appendix A): the exact spherical
 * harmonic coefficients of a band-limited map given on lmax + 2 rings
 * theta_j = pi j / (lmax + 1) (both poles included) with nphi >= 2 mmax + 1
 * equidistant points phi_k = 2 pi k / nphi per ring.  The doubled meridian of
 * 2 lmax + 2 samples determines the field along it; the sin(theta)-weighted
 * integral is taken exactly in Fourier space and folded back onto the rings
 * before the adjoint Legendre step.
 *   map  [ncomp][lmax + 2][nphi] real (prec), ring-major: T, or Q then U;
 *   alm  [ncomp][nalm] complex (prec), overwritten: a_lm, or G then C.
 * Exact up to rounding for maps with band limits (lmax, mmax).  Allocates its own
 * workspace (about (2 mmax + 1) (6 lmax + 6) complex values) and synchronises
 * hip_stream before returning.
 */
int gsht_analysis_minimal(const void *map, int lmax, int mmax, int spin, int nphi,
                          gsht_precision prec, void *alm, void *hip_stream);

/* Thread-local description of the last non-OK status ("" if none).  Host pointer,
 * valid until the next library call on the same thread. */
const char *gsht_last_error(void);

/*
 * Plan API: geometry reuse for many maps on the same points (Sect. 4 notes that
 * many maps are deflected with one set of angles).
 * gsht_plan_create validates the arguments, copies and bin-sorts the points
 * into grid tiles, builds the FFT plans and allocates all workspace; it
 * synchronises hip_stream before returning.  *p is set to NULL on failure.
 * theta/phi are only read during the call.  The oversampling factor is 2; see
 * gsht_plan_create_sigma and gsht_plan_create_tuned for the others.
 */
int gsht_plan_create(gsht_plan **p, int lmax, int mmax, int spin,
                     const double *theta, const double *phi, int64_t npts,
                     double epsilon, gsht_precision prec, void *hip_stream);

/*
 * Plan with a chosen oversampling factor sigma (Sect. 3: about 1.2 to 2; smaller
 * sigma means a smaller torus but a wider kernel for the same epsilon).  sigma must
 * be 2 (what gsht_plan_create uses), 1.5 or 1.25: the kernel's support w and shape
 * beta come from error tables calibrated for these three.  GSHT_EUNSUPPORTED if
 * epsilon needs a wider kernel than the precision's kernels go (16 cells in FP64,
 * 8 in FP32).  Otherwise as gsht_plan_create.
 */
int gsht_plan_create_sigma(gsht_plan **p, int lmax, int mmax, int spin, const double *theta,
                           const double *phi, int64_t npts, double epsilon, gsht_precision prec,
                           double sigma, void *hip_stream);

/*
 * Plan whose oversampling factor sigma and grid tile edge are picked by measurement:
 * builds the plan at every sigma of gsht_plan_create_sigma that reaches epsilon, with
 * tiles of 32, 48 and 64 cells (those whose spreading and interpolation patches fit
 * a workgroup's LDS), times one synthesis + adjoint of each on these points (best of
 * two after a warm-up; zero coefficients and a constant map, since the work does not
 * depend on the values as long as the map is not zero), keeps the fastest and frees
 * the rest.  Holds at most two plans plus one coefficient and one map buffer at a
 * time; a candidate that does not fit is skipped (the sigma = 2, 32-cell plan must
 * build).  Takes a few transforms' time per candidate and, in a new process, the FFT
 * library's set-up for each new length.  gsht_plan_get_info reports the sigma and
 * tile chosen.  (The environment variable GSHT_TILE sets the tile edge of the other
 * plan constructors, for experiments: 16..128 cells, at least w - 1, and a patch
 * within the LDS, else GSHT_EINVAL.)
 */
int gsht_plan_create_tuned(gsht_plan **p, int lmax, int mmax, int spin, const double *theta,
                           const double *phi, int64_t npts, double epsilon, gsht_precision prec,
                           void *hip_stream);

/*
 * New point set for an existing plan (same lmax, mmax, spin, epsilon, precision):
 * theta/phi [npts] FP64 device pointers with npts at most the count the plan was
 * created with.  Only the bin sort is redone (the Legendre tables, column set-up and
 * FFT plans do not depend on the points), so moving points costs a few milliseconds
 * instead of a plan creation: the lensing iterations of Sect. 4 deflect the same
 * pixels differently at every step.  Synchronises hip_stream first (transforms still
 * queued use the old points) and before returning.  GSHT_EINVAL for invalid points
 * (GSHT_EHIP if the sort itself fails): the plan then holds no valid points, and every
 * transform, several-map, derivative and batch call on it, and gsht_plan_get_sort,
 * returns GSHT_EINVAL on the host, before any device work, until a later call of this
 * function succeeds.  Calls on one
 * plan must not overlap with this one, and a graph captured earlier on this plan holds
 * the old sort's buffers: capture again after moving the points.
 */
int gsht_plan_set_points(gsht_plan *p, const double *theta, const double *phi, int64_t npts,
                         void *hip_stream);

/* Synthesis with a plan: alm -> map (layouts as in gsht_synth_general).  Does not
 * allocate and does not synchronise.  Calls on one plan must not overlap.
 * Graph capture: gsht_plan_synth, gsht_plan_adjoint and, once a first call has
 * allocated their buffers, the other plan transforms issue only kernel launches and
 * library FFT launches on hip_stream (no copies, fills or synchronisation), so a
 * caller may capture them into a HIP graph and replay it while the plan lives; a
 * replay reads the buffers captured, at their contents at replay time. */
int gsht_plan_synth(gsht_plan *p, const void *alm, void *map, void *hip_stream);

/*
 * Synthesis of nmaps maps sharing the plan's geometry (Sect. 4: many maps deflected
 * with one set of angles): alm [nmaps][ncomp][nalm] -> map [nmaps][ncomp][npts].
 * Maps are taken in groups whose Legendre step runs in one kernel, the recurrence
 * shared by the group; the later steps run per map.  FP32 plans with lmax <= 8192
 * take groups of 8 to 16 maps through the matrix cores (FP16 hi/lo split products,
 * FP32 accumulation: each map within about 1e-6 relative of its gsht_plan_synth
 * result); remaining maps, and FP64 plans, go in groups of up to four through the
 * FP64 kernel (each map's values as from gsht_plan_synth, up to rounding).  The
 * environment variable GSHT_MANY_MFMA=0 turns the matrix-core path off.  The first
 * call needing a group kind allocates its buffers (FP64 groups: about
 * 4 (nalm 4 ncomp 8 + ncol nd csize) bytes; matrix-core groups: about
 * 16 ncol nd 8 + nalm ncomp 256 bytes), kept until gsht_plan_destroy; later calls do
 * not allocate.  Does not synchronise.
 */
int gsht_plan_synth_many(gsht_plan *p, int nmaps, const void *alm, void *map, void *hip_stream);

/*
 * Adjoint of nmaps maps sharing the plan's geometry (Sect. 2, eq. adjoint, for each
 * map): map [nmaps][ncomp][npts] -> alm [nmaps][ncomp][nalm], each as from
 * gsht_plan_adjoint.  FP32 plans with lmax <= 8192 take groups of 8 to 16 maps
 * through the matrix cores: the spreading and FFT steps run per map, then one kernel
 * forms every map's Legendre sums as FP16 hi/lo split products with FP32
 * accumulation (each map within about 1e-6 relative of its gsht_plan_adjoint
 * result).  Other maps, and FP64 plans, run one at a time.  GSHT_MANY_MFMA=0 turns
 * the matrix-core path off.  The first matrix-core call allocates its buffers (the
 * synthesis group's plus about (mmax + 1) npairs (256 ncomp + 48) + 16 nalm ncomp 16
 * bytes), kept until gsht_plan_destroy.  Does not synchronise.
 */
int gsht_plan_adjoint_many(gsht_plan *p, int nmaps, const void *map, void *alm, void *hip_stream);

/* Launch-shape autotuning: times the Legendre synthesis for 1, 2 and 4 slices of 64
 * ring pairs per wave and the adjoint for every supported (slices, degrees per
 * reduction block) pair on this plan's sizes, and keeps the fastest of each (the
 * results of every shape are the same up to rounding).  Overwrites the plan's
 * internal work buffers only; allocates two small tables; synchronises hip_stream.
 * The chosen shapes are reported by gsht_plan_get_info. */
int gsht_plan_autotune(gsht_plan *p, void *hip_stream);

/* Adjoint with a plan: map -> alm.  Does not allocate and does not synchronise. */
int gsht_plan_adjoint(gsht_plan *p, const void *map, void *alm, void *hip_stream);

/*
 * Gradient-only spin-s transforms (spin > 0 plans; Sect. 4 notes this setting for
 * fields without a curl component): the synthesis of eq. forwardpol with C = 0,
 * and the adjoint's gradient part G only.
 *   glm [1][nalm] complex (prec): G; map [2][npts] real (prec): Q, U.
 * Same results as gsht_plan_synth with C = 0 and as the G block of
 * gsht_plan_adjoint, with about a third fewer Legendre operations (the two spin
 * channels share the products with G).  GSHT_EINVAL for spin-0 plans.  Do not
 * allocate and do not synchronise.
 */
int gsht_plan_synth_grad(gsht_plan *p, const void *glm, void *map, void *hip_stream);
int gsht_plan_adjoint_grad(gsht_plan *p, const void *map, void *glm, void *hip_stream);

/*
 * Derivatives with respect to the point positions (Sect. 2: the lensed map is the
 * unlensed field synthesised at deflected angles, so its dependence on the
 * deflection goes through these derivatives).  With the plan's points:
 *   map     [ncomp][npts] real (prec) or NULL: the synthesis itself;
 *   dtheta  [ncomp][npts] real (prec) or NULL: d map / d theta at each point;
 *   dphi    [ncomp][npts] real (prec) or NULL: d map / d phi at each point.
 * At least one output must be given (else GSHT_EINVAL).  The derivatives come from
 * the same oversampled grid as the synthesis, interpolated with the kernel's
 * derivative; their error relative to the derivative field's norm is of the
 * order of epsilon.  For spin s the components are Q and U in the local
 * (theta, phi) basis, differentiated as functions of the coordinates.
 * Does not allocate and does not synchronise.
 */
int gsht_plan_synth_deriv(gsht_plan *p, const void *alm, void *map, void *dtheta, void *dphi,
                          void *hip_stream);

/*
 * Vector-Jacobian product of the synthesis map = A(alm; theta, phi), for the
 * gradients of a real scalar loss L given gmap = dL/dmap ([ncomp][npts], prec):
 *   galm    [ncomp][nalm] complex (prec) or NULL: dL/dRe(a) + i dL/dIm(a) for every
 *           stored coefficient, which is w_m times the adjoint of gmap (w_0 = 1,
 *           w_m = 2 for m > 0: a stored m > 0 coefficient also sets its -m partner);
 *           entries that the synthesis ignores (Im a_l0, l < spin) are 0;
 *   gtheta  [npts] FP64 or NULL: sum over components of gmap * d map / d theta;
 *   gphi    [npts] FP64 or NULL: the same along phi.
 * alm (the synthesis input) is needed only for gtheta/gphi; the grid is recomputed,
 * not kept from an earlier synthesis.  Does not allocate and does not synchronise.
 */
int gsht_plan_synth_vjp(gsht_plan *p, const void *alm, const void *gmap, void *galm,
                        double *gtheta, double *gphi, void *hip_stream);

/*
 * Vector-Jacobian product of the adjoint alm = A^H(map): given galm =
 * dL/dRe(alm) + i dL/dIm(alm) ([ncomp][nalm] complex, prec), writes
 * gmap = dL/dmap ([ncomp][npts] real, prec), which is the synthesis of galm / w_m.
 * Does not allocate and does not synchronise.
 */
int gsht_plan_adjoint_vjp(gsht_plan *p, const void *galm, void *gmap, void *hip_stream);

/*
 * Lensing geometry (Sect. 2; the deflected-angle formula at the end of Sect. 3).
 *
 * gsht_deflect: for each point n = (theta, phi) and deflection alpha =
 * alpha_theta e_theta + alpha_phi e_phi (|alpha| = a), the point
 *   n' = cos(a) n + (sin(a)/a) (alpha_theta e_theta + alpha_phi e_phi)
 * at distance a along the great circle, and the spin phase chi: the angle by which
 * the basis (e_theta, e_phi) parallel-transported from n to n' along that circle
 * differs from the local basis at n' (chi = beta - beta', the angles the circle
 * makes with e_theta at its ends), so that a spin-s field lenses as
 * sT_len(n) = e^{i s chi} sT_unl(n').
 *   theta, phi   [npts] FP64 device, the undeflected points;
 *   alpha        [2][npts] real (prec): alpha_theta then alpha_phi, as written by a
 *                spin-1 synthesis (Q, U) of sqrt(L(L+1)) (phi_LM + i Omega_LM);
 *   theta_out, phi_out [npts] FP64 out: n' (phi' wrapped to [0, 2 pi));
 *   chi_out      [npts] FP64 out or NULL.
 * Elementwise, stream-ordered; all arithmetic in FP64.
 */
int gsht_deflect(const double *theta, const double *phi, const void *alpha, gsht_precision prec,
                 int64_t npts, double *theta_out, double *phi_out, double *chi_out,
                 void *hip_stream);

/* Vector-Jacobian product of gsht_deflect: given the gradients of a real loss with
 * respect to theta', phi' and chi (FP64 [npts] each, any may be NULL = zero),
 * writes g_alpha [2][npts] (prec), the gradient with respect to (alpha_theta,
 * alpha_phi), from the exact derivatives of the formula above. */
int gsht_deflect_vjp(const double *theta, const void *alpha, gsht_precision prec, int64_t npts,
                     const double *g_theta, const double *g_phi, const double *g_chi,
                     void *g_alpha, void *hip_stream);

/* In place: (Q + iU) <- e^{i sign spin chi} (Q + iU) for map [2][npts] (prec) and
 * chi [npts] FP64; sign is +1 (lensing) or -1 (its adjoint). */
int gsht_spin_phase(void *map, const double *chi, int spin, int sign, gsht_precision prec,
                    int64_t npts, void *hip_stream);

/* Vector-Jacobian product of M = e^{i spin chi} P: given gmap = dL/dM [2][npts]
 * (prec) and the lensed map M (needed only for g_chi), writes
 * g_unrot = dL/dP = e^{-i spin chi} gmap ([2][npts], prec, or NULL) and
 * g_chi = spin (gU MQ - gQ MU) ([npts] FP64, or NULL). */
int gsht_spin_phase_vjp(const void *gmap, const void *lensed, const double *chi, int spin,
                        gsht_precision prec, int64_t npts, void *g_unrot, double *g_chi,
                        void *hip_stream);

/* map_out[c][i] = weights[i] map_in[c][i] for ncomp components ([ncomp][npts] real,
 * prec; weights [npts] FP64; in place allowed): quadrature weights, which turn the
 * adjoint synthesis on a grid into its analysis (Sect. 2: weights added to
 * eq. adjoint approximate the integral over the sphere). */
int gsht_map_weight(const void *map_in, const double *weights, int ncomp, int64_t npts,
                    gsht_precision prec, void *map_out, void *hip_stream);

/* alm_out = sqrt(l (l + 1)) alm_in for ncomp coefficient blocks ([ncomp][nalm]
 * complex, prec; in place allowed): the lensing potential's coefficients become the
 * gradient-mode coefficients of the spin-1 deflection field (eq. deflect). The
 * factor is real, so the same call maps a coefficient gradient back. */
int gsht_alm_lscale(const void *alm_in, void *alm_out, int lmax, int mmax, int ncomp,
                    gsht_precision prec, void *hip_stream);

/* alm_out = f_l alm_in (layout as above) with the real degree factors that map the
 * lensing potential's coefficients onto the fields of Appendix B:
 *   kind 0: sqrt(l (l+1))                   spin-1 deflection (= gsht_alm_lscale),
 *   kind 1: l (l+1) / 2                     spin-0 convergence kappa (omega from the
 *                                           curl potential),
 *   kind 2: sqrt((l-1) l (l+1) (l+2)) / 2   spin-2 shear gamma_1 + i gamma_2,
 * each to be synthesised with the spin given (spin-s sign convention of
 * eq. forwardpol).  GSHT_EINVAL for other kinds. */
int gsht_alm_lfactor(const void *alm_in, void *alm_out, int lmax, int mmax, int ncomp, int kind,
                     gsht_precision prec, void *hip_stream);

/* Magnification determinant |A| of the lensing remapping at each point
 * (Appendix B):  (sin a / a) ((1 - kappa)^2 + omega^2 - gamma^2)
 *   + (cos a - sin a / a) (1 - kappa - cos(2 beta) gamma_1 - sin(2 beta) gamma_2),
 * with a = |alpha| and beta the direction of alpha from e_theta.
 *   alpha [2][npts], kappa [npts], omega [npts] or NULL (= 0), gamma [2][npts]:
 *   real (prec) device maps; det [npts] FP64 out.  Elementwise, stream-ordered. */
int gsht_magnification(const void *alpha, const void *kappa, const void *omega, const void *gamma,
                       gsht_precision prec, int64_t npts, double *det, void *hip_stream);

/* Release a plan and its workspace (NULL is ignored).  Synchronises the device. */
void gsht_plan_destroy(gsht_plan *p);

/*
 * Batches of independent instances (many maps of uneven lmax, spin and point count):
 * a batch owns nstreams (1..16) worker HIP streams of default priority and their
 * events.  gsht_batch_synth / gsht_batch_adjoint run instance i (plans[i] with
 * alms[i] -> maps[i], resp. maps[i] -> alms[i], device pointers, layouts as for the
 * plan calls) on worker stream i mod nstreams, ordered after the work already queued
 * on hip_stream; hip_stream then waits for all of them (event fork and join, no host
 * synchronisation), so small instances overlap on the GPU and a caller may capture a
 * whole batch call into one HIP graph.  The plans must be distinct (each instance
 * uses its plan's work buffers); GSHT_EINVAL otherwise.  On an error in instance i
 * the later instances are not started, the workers are still joined, and the error
 * is returned.  Calls on one batch must not overlap.
 */
typedef struct gsht_batch gsht_batch;
int gsht_batch_create(gsht_batch **b, int nstreams);
int gsht_batch_synth(gsht_batch *b, int n, gsht_plan *const *plans, const void *const *alms,
                     void *const *maps, void *hip_stream);
int gsht_batch_adjoint(gsht_batch *b, int n, gsht_plan *const *plans, const void *const *maps,
                       void *const *alms, void *hip_stream);
void gsht_batch_destroy(gsht_batch *b);

/* Sizes and parameters chosen by a plan (host struct filled by gsht_plan_get_info). */
typedef struct {
    int lmax, mmax, spin, ncomp;
    int64_t npts;
    double epsilon;
    int precision;      /* gsht_precision */
    int ntheta;         /* rings of the equidistant grid, poles included (>= lmax + 2) */
    int ndouble;        /* 2 ntheta - 2: length of the doubled meridian */
    int n1, n2;         /* oversampled torus (theta, phi) */
    int w;              /* kernel support in grid cells */
    double beta;        /* kernel shape: psi(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| < 1 */
    int nrows;          /* torus rows kept (theta in [0, pi] plus the kernel halo) */
    int a_min;          /* torus row index (may be negative, modulo n1) of kept row 0 */
    int tile1, tile2;   /* tile size in grid cells (rows, columns) */
    int ntile1, ntile2; /* tiles per dimension; tile key = (row / tile1) * ntile2 + col / tile2 */
    int64_t nchunks;    /* work items of the interpolation / spreading kernels */
    int64_t workspace_bytes;
    int column_mode;    /* per-column FFT stage: 2 = doubled FFT, deconvolution and theta
                           FFT in one kernel per column (column in LDS), 1 = doubled FFT and
                           deconvolution fused with a separate theta FFT, 0 = separate
                           library FFTs; chosen from the LDS size per workgroup */
    int spread_colors;  /* > 0: spreading runs tile by tile in this many launches of
                           mutually disjoint patches, flushed without atomics; 0: one
                           workgroup per chunk with an atomic flush */
    int syn_r;          /* Legendre synthesis: slices of 64 ring pairs per wave */
    int adj_r, adj_b;   /* Legendre adjoint: slices per wave, degrees per reduction block */
    double sigma;       /* nominal oversampling factor (2, 1.5 or 1.25); n1 and n2 are
                           the FFT-friendly lengths at least about sigma (2 lmax + 1) and
                           sigma (2 mmax + 1) */
    int cell_sort;      /* 1: within a tile, points are ordered by their first kernel cell
                           (see gsht_plan_get_sort); 0: by input order */
} gsht_plan_info;

/* Fill *info from a plan (host only). */
int gsht_plan_get_info(const gsht_plan *p, gsht_plan_info *info);

/*
 * Copy the plan's bin sort out to caller device buffers:
 *   perm        int32 [npts]: perm[k] = input index of the k-th point in sort order
 *               (stable: ties keep input order);
 *   tile_start  int32 [ntile1 * ntile2 + 1]: first sorted position of each tile.
 * Tile key of a point: u = theta * (n1 / (2 pi)), v = phi * (n2 / (2 pi)) (single
 * rounded FP64 products), a0 = ceil(u - w/2), b0 = ceil(v - w/2), r = a0 - a_min,
 * c = b0 mod n2, tile = (r / tile1) * ntile2 + (c / tile2).  With info.cell_sort the
 * sort key is tile * tile1 * tile2 + (r mod tile1) * tile2 + (c mod tile2) (points of
 * a tile by first kernel cell, row-major), otherwise the tile.
 */
int gsht_plan_get_sort(const gsht_plan *p, int32_t *perm, int32_t *tile_start, void *hip_stream);

/*
 * Per-stage timing.  With profiling on, every plan call records HIP events around
 * each stage on hip_stream; gsht_plan_get_stage_times() synchronises on those events
 * and returns, per stage, the total milliseconds and the number of recorded calls
 * since profiling was switched on.  Stage ids are listed by gsht_stage_name().
 */
int gsht_plan_set_profiling(gsht_plan *p, int on);
int gsht_plan_get_stage_times(gsht_plan *p, double *ms, int64_t *count, int nstages);
int gsht_num_stages(void);
const char *gsht_stage_name(int stage);

/*
 * Stage entry point: the "synthesis" and "doubling" steps of Sect. 3 alone.
 * Evaluates F_m(theta_j) = sum_l c_lm sY_lm(theta_j, 0) on the rings
 * theta_j = pi j / (ntheta - 1), j = 0..ntheta-1, and writes the doubled meridian
 *   F[col][j]                       for j < ntheta,
 *   F[col][2 ntheta - 2 - j] = (-1)^(s+m) F[col][j]   for 0 < j < ntheta - 1,
 * where c_lm = a_lm (spin 0) or -(G_lm + i C_lm) (spin > 0, real-field convention
 * for m < 0).  Columns: spin 0 -> col = m, 0..mmax; spin > 0 -> col = m + mmax,
 * -mmax..mmax.  F is complex (complex128 for F64, complex64 for F32),
 * [ncol][2 ntheta - 2].  ntheta >= lmax + 2 is required only for the later steps;
 * here any ntheta >= 2 is accepted.
 */
int gsht_legendre_rings(const void *alm, int lmax, int mmax, int spin, int ntheta,
                        gsht_precision prec, void *F, void *hip_stream);

/*
 * Stage entry point: "undoubling" and "adjoint synthesis" of Sect. 3.  Input F in
 * the doubled layout above; rings 0 < j < ntheta - 1 receive
 *   H_m(theta_j) = F[col][j] + (-1)^(s+m) F[col][2 ntheta - 2 - j],
 * the poles H_m = F[col][j].  Output (overwritten): spin 0 b_lm = sum_j Y_lm(theta_j,0) H_m;
 * spin s: S+ = sum_j sY_lm H_m, S- = sum_j (-s)Y_lm conj(H_{-m}), then the
 * gradient/curl split as in gsht_adjoint_synth_general.
 */
int gsht_legendre_rings_adjoint(const void *F, int lmax, int mmax, int spin, int ntheta,
                                gsht_precision prec, void *alm, void *hip_stream);

/*
 * Allocation-free form of gsht_legendre_rings_adjoint, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, layouts and results; it calls
 * no hipMalloc, hipFree or other allocating routine and does not synchronise.  The
 * Legendre tables, start data and accumulators live in one fixed 64 MiB scratch
 * array per device, held by the library until the process ends; sizes whose tables
 * need more (about 56 nalm bytes for spin > 0, 40 nalm for spin 0) are refused with
 * GSHT_EINVAL before any device work.  Each call rewrites every part of the scratch
 * it reads (start data copied from the host, tables and live-chunk table recomputed,
 * accumulators cleared by a fill kernel).  All calls on one device share its
 * scratch: calls that overlap on one device (other host threads, or other streams
 * still running an earlier call) race and must be serialised by the caller.
 */
int gsht_legendre_rings_adjoint_noalloc(const void *F, int lmax, int mmax, int spin, int ntheta,
                                        gsht_precision prec, void *alm, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GSHT_H */

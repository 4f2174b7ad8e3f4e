// Internal declarations of the gfx950 general-SHT library: the plan object, the
// per-m start data of the Legendre recurrence and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gsht.h"

namespace gsht {

// Start data of the recurrence for one m: the first non-zero degree l0 and, for
// the two channels sigma = +s and sigma = -s, the l-independent factor of
// sY_{l0 m} as (mantissa, binary exponent) and the half-angle exponents:
//   sY_{l0 m}(theta) = mant * 2^ex * sin(theta/2)^a * cos(theta/2)^b.
struct StartInfo {
    int l0;
    int a_p, b_p, ex_p;  // channel +s
    int a_m, b_m, ex_m;  // channel -s
    int pad;
    double mant_p, mant_m;
};

// Device tables of the normalised recurrence p_{l+1} = (a_l x + sigma b_l) p_l - p_{l-1},
// p_l = sY_lm / N_l (identical a_l, b_l, N_l for both channels).
struct LegendreTables {
    double2 *ab = nullptr;     // [nalm]  (a_l, b_l) at idx(l, m), valid for l0 <= l < lmax
    double *norm = nullptr;    // [nalm]  N_l
    StartInfo *start = nullptr;  // [mmax + 1]
    int32_t *lfirst_syn = nullptr;  // [(mmax + 1) * syn_nchunk] first degree a chunk can matter at
    int32_t *lfirst_adj = nullptr;  // [(mmax + 1) * adj_nchunk] same for the adjoint's chunks
};

// One in-LDS FFT of length n (per-column stage): decimation-in-frequency passes of
// the given radices; per pass p (sub-transform length L, stride s = L / r) the
// twiddles w_L^(q j) = exp(-2 pi i q j / L), q = 1..r-1, j < s, stored in the
// plan's precision at tw + twoff[p] + j (r - 1) + q - 1; perm[k] = LDS position of
// frequency k after the last pass (digit reversal).
constexpr int COL_MAXP = 16;

struct ColFFT {
    int n = 0, npass = 0;
    int psh = 31;  // LDS padding: one free slot after every 2^psh elements (31: none)
    int radix[COL_MAXP] = {};
    int twoff[COL_MAXP] = {};
    const void *tw = nullptr;
    const int32_t *perm = nullptr;
};
// Degree of the polynomials that give the FP64 kernel weights of the interior taps.
template <int W>
constexpr int es_pdeg()
{
    return W + 2 > 15 ? W + 2 : 15;
}
inline int es_pdeg_rt(int w) { return w + 2 > 15 ? w + 2 : 15; }

// Position of element i of an in-LDS transform buffer with one padding slot after
// every 2^sh elements (spreads the small-stride passes over the LDS banks), and the
// slots an n-element buffer then takes.
__host__ __device__ inline int lds_pos(int i, int sh) { return i + (i >> sh); }
__host__ __device__ inline int lds_pad_n(int n, int sh) { return sh >= 31 ? n : n + (n >> sh) + 1; }
// Largest LDS buffer a column workgroup may use.
constexpr size_t COL_MAX_BYTES = 163840;
// static LDS of a spreading workgroup beside its patch (work lists and sums)
constexpr size_t SPREAD_STAGE_BYTES = 2048;

enum Stage {
    ST_PREP = 0,
    ST_LEG_SYNTH,
    ST_FFT_D_FWD,
    ST_DECONV_FWD,
    ST_FFT_THETA_INV,
    ST_TRANSPOSE_FWD,
    ST_FFT_PHI_INV,
    ST_INTERP,
    ST_ZERO_GRID,
    ST_SPREAD,
    ST_FFT_PHI_FWD,
    ST_TRANSPOSE_ADJ,
    ST_FFT_THETA_FWD,
    ST_DECONV_ADJ,
    ST_FFT_D_INV,
    ST_LEG_ADJ,
    ST_FINALIZE,
    ST_COLUMN_FWD,
    ST_COLUMN_ADJ,
    ST_INTERP_DERIV,
    ST_COUNT
};

struct FFTPlan {
    rocfft_plan plan = nullptr;
    rocfft_execution_info info = nullptr;
    size_t work_bytes = 0;
};

}  // namespace gsht

struct gsht_plan {
    // problem
    int lmax = 0, mmax = 0, spin = 0, ncomp = 1;
    int64_t npts = 0;
    int64_t npts_cap = 0;  // points the sorted-coordinate buffers hold (set at creation)
    // set only after a complete bin sort and tile colouring; cleared while the points
    // are replaced and left clear when that fails, so no transform runs on a plan
    // whose sort is incomplete
    bool points_ok = false;
    double eps = 0;
    int prec = GSHT_F64;
    // FP64 spreading in the fast fixed-point form (quantisation step 2^-50 of each
    // chunk's value bound; exact form 2^-63)
    bool spread_fast = false;
    // points sorted by tile and, within a tile, by first kernel cell (row, then
    // column); needs ntiles t1 t2 < 2^31 (int32 keys)
    bool cell_sort = false;
    int64_t nalm = 0;
    // grids
    int ntheta = 0, nd = 0, n1 = 0, n2 = 0, w = 0;
    double beta = 0;
    int es_set = 0;  // kernel setting (oversampling factor) index
    int nrows = 0, a_min = 0;
    int t1 = 0, t2 = 0, nt1 = 0, nt2 = 0;
    int tile_req = 0;      // requested tile edge (0: the default 32)
    int64_t ntiles = 0, nchunks = 0;
    int ncol = 0, npairs = 0;
    int syn_r = 2;       // ring pairs per lane, Legendre synthesis (slices of 64)
    int adj_r = 3;       // ring pairs per lane, Legendre adjoint
    int adj_b = 8;       // degrees per reduction block of the adjoint
    int syn_nchunk = 0;  // chunks of 64 * syn_r ring pairs
    int adj_nchunk = 0;  // chunks of 64 * adj_r ring pairs
    int64_t workspace_bytes = 0;
    // device tables
    gsht::LegendreTables leg;
    double *uprep = nullptr;   // prepared coefficients [nalm][2 or 4]
    double *kfac1 = nullptr;   // [lmax + 1] theta deconvolution factor (incl. 1/nd)
    double *kfac2 = nullptr;   // [mmax + 1] phi deconvolution factor
    // geometry
    double *sth = nullptr, *sph = nullptr;  // sorted coordinates
    int32_t *perm = nullptr;                // sorted position -> input index
    int32_t *tile_start = nullptr;          // [ntiles + 1]
    int4 *chunks = nullptr;                 // [nchunks] (tile, begin, end, 0)
    // spreading by tile colour (0 colours = one workgroup per chunk, atomic flush)
    int ncolors = 0;
    int color_start[7] = {};                // items of colour c: [color_start[c], color_start[c+1])
    int2 *tile_items = nullptr;             // (first chunk, number of chunks) per tile
    // work buffers
    void *D = nullptr;     // [ncol][nd] complex
    void *E = nullptr;     // [ncol][n1] complex
    void *G = nullptr;     // complex grid [nrows][n2] (spin > 0) or half spectrum [nrows][n2/2+1]
    void *g = nullptr;     // real grid [nrows][n2] (spin 0 only)
    double *acc = nullptr; // adjoint accumulators [nalm][2 * ncomp]
    double *umulti = nullptr;  // several-map coefficients [nalm][4][2 or 4] (on first use)
    void *Dmulti = nullptr;    // several-map doubled columns [4][ncol][nd] (on first use)
    // matrix-core synthesis of up to 16 maps (FP32 plans, on first use)
    void *Dmfma = nullptr;         // doubled columns [16][ncol][nd]
    void *mfma_tiles = nullptr;    // FP16 coefficient tiles (16 maps)
    int64_t *mfma_boff = nullptr;  // [mmax + 1] first tile block of each m
    float *mfma_scale = nullptr;   // [mmax + 1][16] output scales
    int32_t *mfma_live = nullptr;  // dead-chunk table for slices of 64 ring pairs
    void *mfma_atiles = nullptr;   // FP16 ring-input tiles of the matrix-core adjoint
    float *mfma_ascale = nullptr;  // [mmax + 1][16] their output scales
    double *mfma_acc = nullptr;    // [16][nalm][2 ncomp] adjoint sums of the group
    void *mfma_rstate = nullptr;   // recurrence states of the adjoint's ring slices
    // per-column FFT stage: 0 = rocFFT for both theta transforms, 1 = doubled
    // transform and deconvolution in one kernel (theta transform by rocFFT),
    // 2 = doubled transform, deconvolution and theta transform (split into its
    // even and odd output rows, two transforms of length n1 / 2) in one kernel
    int colmode = 0;
    int lds_psh = 31;         // LDS padding shift of the in-LDS transforms (31: none)
    double *es_poly = nullptr;  // [w][pdeg + 1] interior-tap weight polynomials (FP64 plans)
    gsht::ColFFT cf_d, cf_h;  // lengths nd and n1 / 2
    void *twist = nullptr;    // [n1] exp(-2 pi i k / n1), plan precision (mode 2)
    // FFT plans
    gsht::FFTPlan fD_fwd, fD_inv, fT_inv, fT_fwd, fP_inv, fP_fwd;
    void *fftwork = nullptr;
    size_t fftwork_bytes = 0;
    // profiling
    int profiling = 0;
    hipEvent_t ev[2 * gsht::ST_COUNT] = {};
    int ev_pending[gsht::ST_COUNT] = {};
    double st_ms[gsht::ST_COUNT] = {};
    int64_t st_count[gsht::ST_COUNT] = {};
    std::vector<void *> allocations;
};

namespace gsht {

// ---- Legendre step (legendre.hip) ------------------------------------------
hipError_t launch_leg_tables(const gsht_plan &p, hipStream_t s);
hipError_t launch_leg_live(const gsht_plan &p, hipStream_t s);
hipError_t launch_leg_live_adj(const gsht_plan &p, hipStream_t s);  // adjoint's table only
// mscale multiplies the coefficients (prep) or results (finalize) of every m > 0:
// 1 for the transforms, 1/2 or 2 for the weights w_m of their derivatives.
// grad: gradient-only spin s (C = 0 on input; only G on output).
hipError_t launch_prep_alm(const gsht_plan &p, const void *alm, double mscale, bool grad,
                           hipStream_t s);
hipError_t launch_leg_synth(const gsht_plan &p, void *Dout, bool grad, hipStream_t s);
// several maps sharing the plan: nm in {2, 4}, synthesis slices per lane 1 or 2
hipError_t launch_prep_multi(const gsht_plan &p, const void *alm, int nm, double *u, hipStream_t s);
hipError_t launch_leg_synth_multi(const gsht_plan &p, int nm, const double *u, void *Dout,
                                  size_t dstride, hipStream_t s);
// matrix-core synthesis of nm <= 16 maps (FP32 plans): coefficient tiles and scales,
// the dead-chunk table of its 64-pair chunks, and the Legendre step itself
hipError_t launch_prep_mfma(const gsht_plan &p, const void *alm, int nm, const int64_t *boff,
                            void *tiles, float *oscale, hipStream_t s);
hipError_t launch_leg_live_r1(const gsht_plan &p, int32_t *lfirst1, hipStream_t s);
hipError_t launch_leg_synth_mfma(const gsht_plan &p, int nm, const void *tiles,
                                 const float *oscale, const int64_t *boff,
                                 const int32_t *lfirst1, void *Dout, size_t dstride,
                                 hipStream_t s);
// matrix-core adjoint of nm <= 16 maps (FP32 plans) from their doubled columns
// (map k at Din + k dstride): ring-input tiles, then the sums into accm [nm][nalm][NR]
void adj_mfma_shape(const gsht_plan &p, int &S, int &W);  // W = 0: not possible
size_t adj_mfma_state_bytes(const gsht_plan &p);          // recurrence state buffer
hipError_t launch_prep_adj_mfma(const gsht_plan &p, int nm, const void *Din, size_t dstride,
                                void *tiles, float *oscale, hipStream_t s);
hipError_t launch_leg_adjoint_mfma(const gsht_plan &p, int nm, const void *tiles,
                                   const float *oscale, const int32_t *lfirst1, void *rstate,
                                   double *accm, hipStream_t s);
hipError_t launch_leg_adjoint(const gsht_plan &p, const void *Din, bool grad, hipStream_t s);
hipError_t launch_leg_finalize(const gsht_plan &p, void *alm, double mscale, bool grad,
                               hipStream_t s);

// ---- staging (staging.hip) -------------------------------------------------
hipError_t launch_deconv_fwd(const gsht_plan &p, hipStream_t s);     // D -> E
hipError_t launch_transpose_fwd(const gsht_plan &p, hipStream_t s);  // E -> G
hipError_t launch_transpose_adj(const gsht_plan &p, hipStream_t s);  // G -> E (all rows,
                                                                     // kept rows only if colmode 2)
hipError_t launch_deconv_adj(const gsht_plan &p, hipStream_t s);     // E -> D
hipError_t launch_zero(void *ptr, size_t bytes, hipStream_t s);
hipError_t launch_fill_real(void *ptr, double value, int64_t n, int prec, hipStream_t s);

// ---- per-column FFT stage (colfft.hip) ------------------------------------
hipError_t column_set_lds(const gsht_plan &p);                    // once per plan
int column_half_maxn(int prec);  // largest nd or n1 / 2 of mode 2
int column_max_radix(int prec);  // largest radix the in-LDS transforms are built with
size_t column_lds_bytes(const gsht_plan &p);  // LDS per workgroup of the plan's mode
hipError_t launch_column_fwd(const gsht_plan &p, hipStream_t s);  // D -> E
hipError_t launch_column_adj(const gsht_plan &p, hipStream_t s);  // E -> D

// ---- points (nufft.hip) ----------------------------------------------------
// Bin sort; returns the number of invalid coordinates through *n_invalid (host)
// after synchronising the stream.
hipError_t run_binsort(gsht_plan &p, const double *theta, const double *phi, hipStream_t s,
                       int64_t *n_invalid);
hipError_t build_tile_colors(gsht_plan &p, hipStream_t s);  // after run_binsort
hipError_t launch_interp(const gsht_plan &p, void *map, hipStream_t s);

// ---- minimal-ring analysis (analysis.hip) ------------------------------------
hipError_t launch_pack_rows(const void *map, int spin, int64_t n, int prec, void *P, hipStream_t s);
hipError_t launch_gather_cols(const void *P, int ntheta, int nphi, int nd, int mmax, int spin,
                              int ncol, double scale, int prec, void *D, hipStream_t s);
hipError_t launch_pad_cols(const void *X, int n1, int n2, int kmax, int ncol, double scale,
                           int prec, void *Up, hipStream_t s);
hipError_t launch_trunc_cols(const void *Up, int n1, int n2, int kmax, int ncol, double scale,
                             int prec, void *X, hipStream_t s);
hipError_t launch_weight_cols(void *Up, int n2, int ncol, const double *u, int prec,
                              hipStream_t s);

// ---- lensing geometry (lensing.hip) ------------------------------------------
hipError_t launch_deflect(const double *theta, const double *phi, const void *alpha, int prec,
                          int64_t npts, double *theta_out, double *phi_out, double *chi_out,
                          hipStream_t s);
hipError_t launch_deflect_vjp(const double *theta, const void *alpha, int prec, int64_t npts,
                              const double *g_theta, const double *g_phi, const double *g_chi,
                              void *g_alpha, hipStream_t s);
hipError_t launch_spin_phase(void *map, const double *chi, int spin, int sign, int prec,
                             int64_t npts, hipStream_t s);
hipError_t launch_spin_phase_vjp(const void *g, const void *lensed, const double *chi, int spin,
                                 int prec, int64_t npts, void *g_unrot, double *g_chi,
                                 hipStream_t s);
hipError_t launch_map_weight(const void *in, const double *w, int ncomp, int64_t npts, int prec,
                             void *out, hipStream_t s);
hipError_t launch_alm_lscale(const void *in, int lmax, int mmax, int ncomp, int kind, int prec,
                             void *out, hipStream_t s);
hipError_t launch_magnification(const void *alpha, const void *kappa, const void *omega,
                                const void *gamma, int prec, int64_t npts, double *det,
                                hipStream_t s);
hipError_t launch_interp_deriv(const gsht_plan &p, void *out_map, void *dth, void *dph,
                              const void *gin, double *gth, double *gph, hipStream_t s);
hipError_t launch_spread(const gsht_plan &p, const void *map, hipStream_t s);

}  // namespace gsht

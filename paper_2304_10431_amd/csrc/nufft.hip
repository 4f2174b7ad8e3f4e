// Point side of the general SHT on gfx950: the bin sort of points into grid
// tiles, the type-2 NUFFT interpolation ("NUFFT" step of Sect. 3) and its exact
// transpose, the type-1 spreading (first adjoint step of Sect. 3).
//
// Kernel: psi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| < 1, the exponential of
// semicircle of Barnett et al. (2019) named in Sect. 3.  A point at
// u = theta n1 / (2 pi), v = phi n2 / (2 pi) touches the w x w cells
// a0 + i, b0 + j with a0 = ceil(u - w/2), b0 = ceil(v - w/2), with weights
// psi((u - a0 - i) 2/w) psi((v - b0 - j) 2/w).  Offsets are formed in FP64 and
// only then rounded to the working precision.
//
// Points are processed in tile order: every work item ("chunk") holds at most
// CHUNK consecutive sorted points of one tile, and stages that tile's grid patch
// (tile plus a w - 1 halo) in LDS.  Spreading accumulates into the LDS patch with
// fixed-point integer LDS atomics and then flushes it to the grid with global atomics.
#include <cstdlib>
#include <vector>

#include "gsht_internal.hpp"

#include <algorithm>
#include <type_traits>

namespace gsht {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 16;  // per thread
constexpr int SORT_BLOCK = SORT_THREADS * SORT_ITEMS;
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int CHUNK = 512;
constexpr int NUFFT_THREADS = 256;
// Accepted |phi| (radians); beyond it the FP64 cell offsets would lose too much accuracy.
constexpr double PHI_MAX = 1048576.0;

// ---- keys ------------------------------------------------------------------------

struct KeyParams {
    double c1, c2, half;
    int a_min, n2, t1, t2, nt2, nrows, w;
    int cells;  // key within the tile too: tile t1 t2 + row t2 + column (cell order)
};

// First kernel cell of a point.  u = theta c1 and v = phi c2 are single-rounded
// products and u - w/2, v - w/2 single-rounded differences (contraction into an
// FMA is switched off), so the cells match a plain FP64 evaluation bit for bit;
// the column is reduced modulo n2 in exact integer arithmetic.  Used by both the
// key computation and the interpolation/spreading kernels.
struct Cell {
    double u, v, a0, b0;  // a0, b0 integer valued
    int r0, bi;           // kept-row offset (clamped) and column in [0, n2)
};

__device__ inline Cell point_cell(double th, double ph, double c1, double c2, double half,
                                  int a_min, int n2, int nrows, int w)
{
#pragma clang fp contract(off)
    Cell c;
    c.u = th * c1;
    c.v = ph * c2;
    c.a0 = ceil(c.u - half);
    c.b0 = ceil(c.v - half);
    int64_t r0 = (int64_t)c.a0 - a_min;
    r0 = r0 < 0 ? 0 : r0;
    r0 = r0 > nrows - w ? nrows - w : r0;
    c.r0 = (int)r0;
    if (c.b0 >= 0.0 && c.b0 < (double)n2) {
        c.bi = (int)c.b0;
    } else {
        int64_t b = (int64_t)c.b0 % n2;  // |b0| < 2^62 (|phi| is bounded on entry)
        c.bi = (int)(b < 0 ? b + n2 : b);
    }
    return c;
}

__global__ void keys_kernel(const double *__restrict__ theta, const double *__restrict__ phi,
                            int64_t npts, KeyParams kp, int32_t *__restrict__ keys,
                            int32_t *__restrict__ vals, unsigned long long *__restrict__ n_invalid)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts)
        return;
    const double th = theta[i], ph = phi[i];
    int key = 0;
    const bool ok = (th >= 0.0) && (th <= 3.141592653589793) && (fabs(ph) <= PHI_MAX);
    if (!ok) {
        atomicAdd(n_invalid, 1ull);
    } else {
        const Cell c = point_cell(th, ph, kp.c1, kp.c2, kp.half, kp.a_min, kp.n2, kp.nrows, kp.w);
        key = (c.r0 / kp.t1) * kp.nt2 + c.bi / kp.t2;
        if (kp.cells)
            key = key * (kp.t1 * kp.t2) + (c.r0 % kp.t1) * kp.t2 + c.bi % kp.t2;
    }
    keys[i] = key;
    vals[i] = (int32_t)i;
}

// ---- stable LSD radix sort of (key, value) pairs -------------------------------

__global__ __launch_bounds__(SORT_THREADS) void radix_hist_kernel(const int32_t *__restrict__ keys,
                                                                  int64_t n, int shift, int nblocks,
                                                                  int32_t *__restrict__ counts)
{
    __shared__ int h[RADIX];
    for (int d = threadIdx.x; d < RADIX; d += SORT_THREADS)
        h[d] = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * SORT_BLOCK;
    for (int it = 0; it < SORT_ITEMS; ++it) {
        const int64_t i = b0 + it * SORT_THREADS + threadIdx.x;
        if (i < n)
            atomicAdd(&h[(keys[i] >> shift) & (RADIX - 1)], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < RADIX; d += SORT_THREADS)
        counts[(size_t)d * nblocks + blockIdx.x] = h[d];
}

// Exclusive scan helpers (int32, total < 2^31).
constexpr int SCAN_TILE = 1024;

__global__ __launch_bounds__(SCAN_TILE) void scan_tile_sums(const int32_t *__restrict__ in, int64_t n,
                                                            int32_t *__restrict__ sums)
{
    __shared__ int s[SCAN_TILE];
    const int64_t i = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
    s[threadIdx.x] = (i < n) ? in[i] : 0;
    __syncthreads();
    for (int d = SCAN_TILE / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d)
            s[threadIdx.x] += s[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        sums[blockIdx.x] = s[0];
}

// Single block: exclusive scan of the tile sums in place (sequential over
// groups of SCAN_TILE, each group scanned in LDS).
__global__ __launch_bounds__(SCAN_TILE) void scan_sums_kernel(int32_t *__restrict__ sums, int64_t n)
{
    __shared__ int s[SCAN_TILE];
    int carry = 0;
    for (int64_t g = 0; g < n; g += SCAN_TILE) {
        const int64_t i = g + threadIdx.x;
        const int v = (i < n) ? sums[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < SCAN_TILE; d <<= 1) {
            const int t = ((int)threadIdx.x >= d) ? s[threadIdx.x - d] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n)
            sums[i] = carry + s[threadIdx.x] - v;
        const int tot = s[SCAN_TILE - 1];
        __syncthreads();
        carry += tot;
    }
}

__global__ __launch_bounds__(SCAN_TILE) void scan_apply_kernel(const int32_t *__restrict__ in, int64_t n,
                                                               const int32_t *__restrict__ sums,
                                                               int32_t *__restrict__ out)
{
    __shared__ int s[SCAN_TILE];
    const int64_t i = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
    const int v = (i < n) ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < SCAN_TILE; d <<= 1) {
        const int t = ((int)threadIdx.x >= d) ? s[threadIdx.x - d] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n)
        out[i] = sums[blockIdx.x] + s[threadIdx.x] - v;
}

static hipError_t exclusive_scan(const int32_t *in, int64_t n, int32_t *out, int32_t *tmp,
                                 hipStream_t s)
{
    const int64_t ntile = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)ntile), dim3(SCAN_TILE), 0, s, in, n, tmp);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(SCAN_TILE), 0, s, tmp, ntile);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)ntile), dim3(SCAN_TILE), 0, s, in, n, tmp,
                       out);
    return hipGetLastError();
}

// Stable scatter: items of a block are ranked in input order.  Each round takes
// SORT_THREADS consecutive items; within a wave, lanes with equal digits are found
// with one ballot per digit bit.
__global__ __launch_bounds__(SORT_THREADS) void radix_scatter_kernel(
    const int32_t *__restrict__ kin, const int32_t *__restrict__ vin, int64_t n, int shift,
    int nblocks, const int32_t *__restrict__ offsets, int32_t *__restrict__ kout,
    int32_t *__restrict__ vout)
{
    constexpr int NW = SORT_THREADS / 64;
    __shared__ int run[RADIX];
    __shared__ int wcnt[NW][RADIX];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int d = tid; d < RADIX; d += SORT_THREADS)
        run[d] = offsets[(size_t)d * nblocks + blockIdx.x];
    const int64_t b0 = (int64_t)blockIdx.x * SORT_BLOCK;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int it = 0; it < SORT_ITEMS; ++it) {
        for (int d = tid; d < NW * RADIX; d += SORT_THREADS)
            (&wcnt[0][0])[d] = 0;
        __syncthreads();
        const int64_t i = b0 + (int64_t)it * SORT_THREADS + tid;
        const bool valid = i < n;
        const int k = valid ? kin[i] : 0;
        const int dg = valid ? ((k >> shift) & (RADIX - 1)) : 0;
        unsigned long long eq = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; ++b) {
            const unsigned long long bb = __ballot(valid && ((dg >> b) & 1));
            eq &= ((dg >> b) & 1) ? bb : ~bb;
        }
        const int rank_w = __popcll(eq & lt);
        if (valid && rank_w == 0)
            wcnt[wv][dg] = __popcll(eq);
        __syncthreads();
        if (valid) {
            int off = run[dg];
            for (int w2 = 0; w2 < wv; ++w2)
                off += wcnt[w2][dg];
            const int dst = off + rank_w;
            if (dst >= 0 && dst < n) {
                kout[dst] = k;
                vout[dst] = vin[i];
            }
        }
        __syncthreads();
        for (int d = tid; d < RADIX; d += SORT_THREADS) {
            int t = 0;
            for (int w2 = 0; w2 < NW; ++w2)
                t += wcnt[w2][d];
            run[d] += t;
        }
        __syncthreads();
    }
}

// tile_start[t] = first sorted position whose tile (key / cpt, cpt keys per tile) is >= t.
__global__ void tile_start_kernel(const int32_t *__restrict__ skeys, int64_t n, int64_t ntiles,
                                  int cpt, int32_t *__restrict__ start)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > n)
        return;
    const int64_t lo = (p == 0) ? 0 : (int64_t)(skeys[p - 1] / cpt) + 1;
    const int64_t hi = (p == n) ? ntiles : (int64_t)(skeys[p] / cpt);
    for (int64_t t = lo; t <= hi; ++t)
        start[t] = (int32_t)p;
}

__global__ void chunk_count_kernel(const int32_t *__restrict__ start, int64_t ntiles,
                                   int32_t *__restrict__ cnt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles)
        return;
    const int c = start[t + 1] - start[t];
    cnt[t] = (c + CHUNK - 1) / CHUNK;
}

__global__ void chunk_fill_kernel(const int32_t *__restrict__ start, const int32_t *__restrict__ coff,
                                  int64_t ntiles, int4 *__restrict__ chunks)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles)
        return;
    const int b = start[t], e = start[t + 1];
    int o = coff[t];
    for (int c = b; c < e; c += CHUNK)
        chunks[o++] = make_int4((int)t, c, (c + CHUNK < e) ? c + CHUNK : e, 0);
}

__global__ void gather_coords_kernel(const double *__restrict__ theta, const double *__restrict__ phi,
                                     const int32_t *__restrict__ perm, int64_t n,
                                     double *__restrict__ sth, double *__restrict__ sph)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    const int32_t i = perm[p];
    sth[p] = theta[i];
    sph[p] = phi[i];
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t run_binsort(gsht_plan &p, const double *theta, const double *phi, hipStream_t s,
                       int64_t *n_invalid)
{
    const int64_t n = p.npts;
    hipError_t e;
    *n_invalid = 0;
    // scratch: keys/vals double buffers, counts, scan temp
    const int64_t nblocks = (n + SORT_BLOCK - 1) / SORT_BLOCK;
    const int64_t ncount = nblocks * RADIX;
    const int64_t nscan = (std::max(ncount, p.ntiles) + SCAN_TILE - 1) / SCAN_TILE + 1;
    int32_t *k0 = nullptr, *k1 = nullptr, *v0 = nullptr, *v1 = nullptr, *cnt = nullptr,
            *tmp = nullptr;
    unsigned long long *inval = nullptr;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const size_t ncnt = (size_t)std::max<int64_t>(std::max(ncount, p.ntiles + 1), 1);
    if ((e = hipMalloc(&k0, nn * 4)) != hipSuccess) goto out;
    if ((e = hipMalloc(&k1, nn * 4)) != hipSuccess) goto out;
    if ((e = hipMalloc(&v0, nn * 4)) != hipSuccess) goto out;
    if ((e = hipMalloc(&v1, nn * 4)) != hipSuccess) goto out;
    if ((e = hipMalloc(&cnt, ncnt * 4)) != hipSuccess) goto out;
    if ((e = hipMalloc(&tmp, (size_t)nscan * 4 + 16)) != hipSuccess) goto out;
    if ((e = hipMalloc(&inval, sizeof(unsigned long long))) != hipSuccess) goto out;
    if ((e = launch_zero(inval, sizeof(unsigned long long), s)) != hipSuccess) goto out;
    if (n > 0) {
        KeyParams kp;
        kp.c1 = (double)p.n1 / (2.0 * 3.141592653589793);
        kp.c2 = (double)p.n2 / (2.0 * 3.141592653589793);
        kp.half = 0.5 * (double)p.w;
        kp.a_min = p.a_min;
        kp.n2 = p.n2;
        kp.t1 = p.t1;
        kp.t2 = p.t2;
        kp.nt2 = p.nt2;
        kp.nrows = p.nrows;
        kp.w = p.w;
        kp.cells = p.cell_sort ? 1 : 0;
        hipLaunchKernelGGL(keys_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, theta, phi, n, kp, k0,
                           v0, inval);
        if ((e = hipGetLastError()) != hipSuccess) goto out;
        const int64_t nkeys = p.ntiles * (p.cell_sort ? (int64_t)p.t1 * p.t2 : 1);
        int bits = 1;
        while (bits < 31 && ((int64_t)1 << bits) < nkeys)
            ++bits;
        for (int shift = 0; shift < bits; shift += RADIX_BITS) {
            hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nblocks), dim3(SORT_THREADS), 0, s,
                               k0, n, shift, (int)nblocks, cnt);
            if ((e = exclusive_scan(cnt, ncount, cnt, tmp, s)) != hipSuccess) goto out;
            hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nblocks), dim3(SORT_THREADS), 0,
                               s, k0, v0, n, shift, (int)nblocks, cnt, k1, v1);
            if ((e = hipGetLastError()) != hipSuccess) goto out;
            std::swap(k0, k1);
            std::swap(v0, v1);
        }
    }
    hipLaunchKernelGGL(tile_start_kernel, dim3(nblk(n + 1, 256)), dim3(256), 0, s, k0, n, p.ntiles,
                       p.cell_sort ? p.t1 * p.t2 : 1, p.tile_start);
    if ((e = hipMemcpyAsync(p.perm, v0, nn * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess) goto out;
    if (n > 0) {
        hipLaunchKernelGGL(gather_coords_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, theta, phi,
                           p.perm, n, p.sth, p.sph);
    }
    // chunk list
    hipLaunchKernelGGL(chunk_count_kernel, dim3(nblk(p.ntiles, 256)), dim3(256), 0, s, p.tile_start,
                       p.ntiles, cnt);
    if ((e = exclusive_scan(cnt, p.ntiles, cnt, tmp, s)) != hipSuccess) goto out;
    {
        int32_t last_off = 0, last_cnt = 0, tot;
        unsigned long long hinv = 0;
        // total chunks = offset of the last tile + its chunk count
        int32_t ends[2];
        if ((e = hipMemcpyAsync(&last_off, cnt + (p.ntiles - 1), 4, hipMemcpyDeviceToHost, s)) !=
            hipSuccess) goto out;
        if ((e = hipMemcpyAsync(ends, p.tile_start + (p.ntiles - 1), 8, hipMemcpyDeviceToHost, s)) !=
            hipSuccess) goto out;
        if ((e = hipMemcpyAsync(&hinv, inval, sizeof(hinv), hipMemcpyDeviceToHost, s)) != hipSuccess)
            goto out;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) goto out;
        last_cnt = (ends[1] - ends[0] + CHUNK - 1) / CHUNK;
        tot = last_off + last_cnt;
        *n_invalid = (int64_t)hinv;
        p.nchunks = tot;
        if (tot > 0) {
            if ((e = hipMalloc(&p.chunks, (size_t)tot * sizeof(int4))) != hipSuccess) goto out;
            p.allocations.push_back(p.chunks);
            hipLaunchKernelGGL(chunk_fill_kernel, dim3(nblk(p.ntiles, 256)), dim3(256), 0, s,
                               p.tile_start, cnt, p.ntiles, p.chunks);
            if ((e = hipGetLastError()) != hipSuccess) goto out;
        }
        e = hipStreamSynchronize(s);
    }
out:  // scratch of the sort; a failed free cannot change the result
    (void)hipFree(k0);
    (void)hipFree(k1);
    (void)hipFree(v0);
    (void)hipFree(v1);
    (void)hipFree(cnt);
    (void)hipFree(tmp);
    (void)hipFree(inval);
    return e;
}

// Spreading work by tile colour: tile (tr, tc) gets colour (tr & 1) + 2 cc with
// cc = tc & 1, except that with an odd number of tile columns the last column (a
// neighbour of column 0 across phi = 0) gets cc = 2.  Tiles of one colour are then
// at least two tiles apart, and with tiles at least W - 1 cells wide their patches
// are disjoint.  Needs at least two tile columns; otherwise ncolors stays 0 and the
// spreading flushes with atomics.  GSHT_SPREAD_COLORS=0 forces the atomic flush.
hipError_t build_tile_colors(gsht_plan &p, hipStream_t s)
{
    p.ncolors = 0;
    const char *env = getenv("GSHT_SPREAD_COLORS");
    // A patch spans its tile plus w - 1 cells to the right, modulo n2 in phi.  It must
    // not wrap onto itself (t2 + w - 1 <= n2), and with an even number of tile
    // columns the last (possibly narrower) column lies between two colour-0 columns
    // across the wrap, so it must be at least w - 1 cells wide.
    const int last = p.n2 - (p.nt2 - 1) * p.t2;
    if ((env && atoi(env) == 0) || p.nchunks == 0 || p.nt2 < 2 || p.t1 < p.w - 1 ||
        p.t2 < p.w - 1 || p.t2 + p.w - 1 > p.n2 || (p.nt2 % 2 == 0 && last < p.w - 1))
        return hipSuccess;
    std::vector<int4> ck((size_t)p.nchunks);
    hipError_t e = hipMemcpyAsync(ck.data(), p.chunks, sizeof(int4) * ck.size(),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return e;
    const int ncc = (p.nt2 % 2 == 0) ? 2 : 3;
    const int ncol = 2 * ncc;
    std::vector<std::vector<int2>> lists((size_t)ncol);
    for (size_t i = 0; i < ck.size();) {
        size_t j = i + 1;
        while (j < ck.size() && ck[j].x == ck[i].x)
            ++j;
        const int t = ck[i].x, tr = t / p.nt2, tc = t - tr * p.nt2;
        const int cc = (ncc == 3 && tc == p.nt2 - 1) ? 2 : (tc & 1);
        lists[(size_t)((tr & 1) + 2 * cc)].push_back(make_int2((int)i, (int)(j - i)));
        i = j;
    }
    std::vector<int2> items;
    items.reserve(ck.size());
    p.color_start[0] = 0;
    for (int c = 0; c < ncol; ++c) {
        items.insert(items.end(), lists[(size_t)c].begin(), lists[(size_t)c].end());
        p.color_start[c + 1] = (int)items.size();
    }
    if ((e = hipMalloc(&p.tile_items, sizeof(int2) * items.size())) != hipSuccess)
        return e;
    p.allocations.push_back(p.tile_items);
    if ((e = hipMemcpyAsync(p.tile_items, items.data(), sizeof(int2) * items.size(),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
        return e;
    p.ncolors = ncol;
    return hipSuccess;
}

// ---- interpolation and spreading ------------------------------------------------

template <typename T> struct cpl;
template <> struct cpl<float> { using type = float2; };
template <> struct cpl<double> { using type = double2; };

template <typename T> __device__ inline T es_kernel(T z, T beta);
template <> __device__ inline float es_kernel<float>(float z, float beta)
{
    return __expf(beta * (sqrtf(fmaxf(0.0f, 1.0f - z * z)) - 1.0f));
}
template <> __device__ inline double es_kernel<double>(double z, double beta)
{
    return exp(beta * (sqrt(fmax(0.0, 1.0 - z * z)) - 1.0));
}

struct GridGeom {
    const double *poly;  // FP64 interior-tap kernel polynomials (or null), see point_weights
    double c1, c2, half;
    int a_min, n2, stride, nrows, t1, t2, nt2;
    int ps;      // row stride of a tile's LDS patch in cells (t2 + w - 1)
    int64_t npts;
};

// Cell indices and kernel weights of one point, relative to a patch origin.
// POLY: FP64 interior taps by polynomial when the plan has them (interpolation; the
// spreading kernels keep the exact formula, which measured faster there).
template <typename T, int W, bool POLY = false>
__device__ inline void point_weights(double th, double ph, const GridGeom &g, int row0, int col0,
                                     T beta, int &lr, int &lc, T (&wx)[W], T (&wy)[W])
{
    const Cell c = point_cell(th, ph, g.c1, g.c2, g.half, g.a_min, g.n2, g.nrows, W);
    const double dx = c.u - c.a0, dy = c.v - c.b0;  // in (w/2 - 1, w/2]
    lr = c.r0 - row0;
    lc = c.bi - col0;
    const T sc = (T)(2.0 / W);
    const T fx = (T)dx, fy = (T)dy;
    if constexpr (POLY && std::is_same<T, double>::value) {
        if (g.poly != nullptr) {
            // FP64: the two edge taps (whose interval ends at the kernel's square-root
            // edge) exactly; each interior tap i by its polynomial in y = 2 dx - W + 1
            // (the offset mapped to (-1, 1]), fitted on the host to ~1e-15 absolute.
            constexpr int PD = es_pdeg<W>();
            const double yx = 2.0 * dx - (double)(W - 1), yy = 2.0 * dy - (double)(W - 1);
            wx[0] = es_kernel<T>(fx * sc, beta);
            wy[0] = es_kernel<T>(fy * sc, beta);
            wx[W - 1] = es_kernel<T>((fx - (T)(W - 1)) * sc, beta);
            wy[W - 1] = es_kernel<T>((fy - (T)(W - 1)) * sc, beta);
#pragma unroll
            for (int i = 1; i < W - 1; ++i) {
                const double *c = g.poly + i * (PD + 1);
                double px = c[PD], py = c[PD];
#pragma unroll
                for (int k = PD - 1; k >= 0; --k) {
                    px = fma(px, yx, c[k]);
                    py = fma(py, yy, c[k]);
                }
                wx[i] = px;
                wy[i] = py;
            }
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < W; ++i) {
        wx[i] = es_kernel<T>((fx - (T)i) * sc, beta);
        wy[i] = es_kernel<T>((fy - (T)i) * sc, beta);
    }
}

// One workgroup per chunk, or (items non-null) per tile: items[b] = (first chunk, number
// of chunks) of one tile, whose points are then one contiguous range, and the patch is
// loaded once for all of them.
template <typename T, int W, bool CPLX>
__global__ __launch_bounds__(NUFFT_THREADS) void interp_kernel(
    const int4 *__restrict__ chunks, const int2 *__restrict__ items,
    const double *__restrict__ sth, const double *__restrict__ sph,
    const int32_t *__restrict__ perm, const void *__restrict__ gridv, GridGeom g, T beta,
    T *__restrict__ out)
{
    using C = typename cpl<T>::type;
    using V = typename std::conditional<CPLX, C, T>::type;
    extern __shared__ unsigned char smem_raw[];
    V *patch = reinterpret_cast<V *>(smem_raw);
    const V *grid = reinterpret_cast<const V *>(gridv);
    int4 ck;
    if (items != nullptr) {
        const int2 it = items[blockIdx.x];
        ck = chunks[it.x];
        ck.z = chunks[it.x + it.y - 1].z;
    } else {
        ck = chunks[blockIdx.x];
    }
    const int tr = ck.x / g.nt2, tc = ck.x - (ck.x / g.nt2) * g.nt2;
    const int row0 = tr * g.t1, col0 = tc * g.t2;
    const int PR = g.t1 + W - 1, PC = g.t2 + W - 1;
    for (int idx = threadIdx.x; idx < PR * PC; idx += NUFFT_THREADS) {
        const int pr = idx / PC, pc = idx - (idx / PC) * PC;
        const int r = row0 + pr;
        int c = col0 + pc;
        while (c >= g.n2)  // patches may span the torus more than once when n2 is small
            c -= g.n2;
        V v{};
        if (r < g.nrows)
            v = grid[(size_t)r * g.stride + c];
        patch[pr * g.ps + pc] = v;
    }
    __syncthreads();
    for (int p = ck.y + threadIdx.x; p < ck.z; p += NUFFT_THREADS) {
        T wx[W], wy[W];
        int lr, lc;
        point_weights<T, W, true>(sth[p], sph[p], g, row0, col0, beta, lr, lc, wx, wy);
        if (lr < 0 || lr >= g.t1 || lc < 0 || lc >= g.t2)
            continue;  // cannot happen for points sorted by the same arithmetic
        T ar = 0, ai = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const V *rowp = patch + (lr + i) * g.ps + lc;
            T sr = 0, si = 0;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                if constexpr (CPLX) {
                    const C v = rowp[j];
                    sr = fma(wy[j], v.x, sr);
                    si = fma(wy[j], v.y, si);
                } else {
                    sr = fma(wy[j], rowp[j], sr);
                }
            }
            ar = fma(wx[i], sr, ar);
            if constexpr (CPLX)
                ai = fma(wx[i], si, ai);
        }
        const int32_t dst = perm[p];
        out[dst] = ar;
        if constexpr (CPLX)
            out[g.npts + dst] = ai;
    }
}

// Kernel weight and its derivative with respect to the point's cell coordinate at
// z = 2 (u - a) / W:  d/du exp(beta (sqrt(1 - z^2) - 1)) = -beta z / sqrt(1 - z^2)
// * (2 / W) times the weight (taken as 0 at |z| = 1, where the kernel's value is
// e^-beta and its slope unbounded).
template <typename T, int W>
__device__ inline void es_weight_d(T z, T beta, T &wv, T &dv)
{
    const T q = sqrt(fmax((T)0, (T)1 - z * z));
    wv = exp(beta * (q - (T)1));
    dv = q > (T)0 ? -beta * z / q * (T)(2.0 / W) * wv : (T)0;
}

// Type-2 interpolation of the map's first derivatives: with the patch values G,
//   f = sum G w_i w_j,  df/du = sum G w'_i w_j,  df/dv = sum G w_i w'_j,
// d/dtheta = (N1 / 2 pi) d/du and d/dphi = (N2 / 2 pi) d/dv.  Without VJP the
// derivative maps are written ([ncomp][npts], any of map / dth / dph may be null);
// with VJP the products with the incoming map gradient gin are summed over the
// components and written in FP64 to gth / gph ([npts], either may be null).
template <typename T, int W, bool CPLX, bool VJP>
__global__ __launch_bounds__(NUFFT_THREADS) void interp_deriv_kernel(
    const int4 *__restrict__ chunks, const double *__restrict__ sth, const double *__restrict__ sph,
    const int32_t *__restrict__ perm, const void *__restrict__ gridv, GridGeom g, T beta,
    T *__restrict__ map, T *__restrict__ dth, T *__restrict__ dph, const T *__restrict__ gin,
    double *__restrict__ gth, double *__restrict__ gph)
{
    using C = typename cpl<T>::type;
    using V = typename std::conditional<CPLX, C, T>::type;
    constexpr int NC = CPLX ? 2 : 1;
    extern __shared__ unsigned char smem_raw[];
    V *patch = reinterpret_cast<V *>(smem_raw);
    const V *grid = reinterpret_cast<const V *>(gridv);
    const int4 ck = chunks[blockIdx.x];
    const int tr = ck.x / g.nt2, tc = ck.x - (ck.x / g.nt2) * g.nt2;
    const int row0 = tr * g.t1, col0 = tc * g.t2;
    const int PR = g.t1 + W - 1, PC = g.t2 + W - 1;
    for (int idx = threadIdx.x; idx < PR * PC; idx += NUFFT_THREADS) {
        const int pr = idx / PC, pc = idx - (idx / PC) * PC;
        const int r = row0 + pr;
        int c = col0 + pc;
        while (c >= g.n2)  // patches may span the torus more than once when n2 is small
            c -= g.n2;
        V v{};
        if (r < g.nrows)
            v = grid[(size_t)r * g.stride + c];
        patch[pr * g.ps + pc] = v;
    }
    __syncthreads();
    const T cu = (T)g.c1, cv = (T)g.c2;
    const T sc = (T)(2.0 / W);
    for (int p = ck.y + threadIdx.x; p < ck.z; p += NUFFT_THREADS) {
        const Cell cell = point_cell(sth[p], sph[p], g.c1, g.c2, g.half, g.a_min, g.n2, g.nrows, W);
        const int lr = cell.r0 - row0, lc = cell.bi - col0;
        if (lr < 0 || lr >= g.t1 || lc < 0 || lc >= g.t2)
            continue;  // cannot happen for points sorted by the same arithmetic
        const T fx = (T)(cell.u - cell.a0), fy = (T)(cell.v - cell.b0);  // in (w/2 - 1, w/2]
        T wy[W], dwy[W];
#pragma unroll
        for (int j = 0; j < W; ++j)
            es_weight_d<T, W>((fy - (T)j) * sc, beta, wy[j], dwy[j]);
        T f[NC] = {}, fu[NC] = {}, fv[NC] = {};
#pragma unroll 1
        for (int i = 0; i < W; ++i) {
            T wxi, dwxi;
            es_weight_d<T, W>((fx - (T)i) * sc, beta, wxi, dwxi);
            const V *rowp = patch + (lr + i) * g.ps + lc;
            T s0[NC] = {}, s1[NC] = {};
#pragma unroll
            for (int j = 0; j < W; ++j) {
                if constexpr (CPLX) {
                    const C v = rowp[j];
                    s0[0] = fma(wy[j], v.x, s0[0]);
                    s0[1] = fma(wy[j], v.y, s0[1]);
                    s1[0] = fma(dwy[j], v.x, s1[0]);
                    s1[1] = fma(dwy[j], v.y, s1[1]);
                } else {
                    s0[0] = fma(wy[j], rowp[j], s0[0]);
                    s1[0] = fma(dwy[j], rowp[j], s1[0]);
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                f[c] = fma(wxi, s0[c], f[c]);
                fu[c] = fma(dwxi, s0[c], fu[c]);
                fv[c] = fma(wxi, s1[c], fv[c]);
            }
        }
        const int32_t dst = perm[p];
        if constexpr (VJP) {
            double at = 0.0, ap = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double gc = (double)gin[c * g.npts + dst];
                at += gc * (double)(cu * fu[c]);
                ap += gc * (double)(cv * fv[c]);
            }
            if (gth)
                gth[dst] = at;
            if (gph)
                gph[dst] = ap;
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (map)
                    map[c * g.npts + dst] = f[c];
                if (dth)
                    dth[c * g.npts + dst] = cu * fu[c];
                if (dph)
                    dph[c * g.npts + dst] = cv * fv[c];
            }
        }
    }
}

// Rounding by the magic constant M = 1.5 2^52: for |x| < 2^51 the double x + M has
// exponent 52, so its bits read as a 64-bit integer are KM + round(x) (round to
// nearest even), with KM = bits(M) = 0x4338000000000000, which is zero below bit 51.
// fma(a, b, M) rounds the exact product a b once.  The low 32 bits are round(x) mod
// 2^32, and a sum of such words carries the KM terms only in bits 51 and up.
constexpr double QMAGIC = 6755399441055744.0;
constexpr unsigned int QMAGIC_HI = 0x43380000u;  // KMhi: bits 32..63 of KM
__device__ inline unsigned long long qbits(double a, double b)
{
    return (unsigned long long)__double_as_longlong(fma(a, b, QMAGIC));
}

// Fixed-point accumulator of the spreading patch: on gfx950 integer LDS atomic adds
// run 3.6x (u32) / 2x (u64) faster than FP64 ones and 26x faster than FP32 ones.
// quant(a, b) is round(a b) in the accumulator's word; total(t) reads a cell sum back.
// FP32 grids: 32-bit words, step S / 2^31.  FP64 grids, exact form (FQ = false):
// 64-bit words, step S / 2^63, converted by the library's double -> int64 rounding.
// FP64, fast form (FQ = true): step S / 2^50, every cell sum stays within 2^50 in
// magnitude, so the low 51 bits of the sum of magic-rounded words are the sum
// itself (sign-extended) whatever the KM terms did above them: one FMA per word.
template <typename T, bool FQ> struct SpreadAcc;
// Packed FP32 cell word from the magic-rounded bits of Re (taken with M - 2^32 KMhi)
// and Im: bi + (br << 32), formed as its two 32-bit halves (no carry crosses them):
// one 32-bit add on the high half (written as such, since the compiler otherwise
// rebuilds the 64-bit form with an extra move).
__device__ inline unsigned long long pack_word(unsigned long long br, unsigned long long bi)
{
    uint2 w;
    w.x = (unsigned int)bi;
    asm("v_add_u32 %0, %1, %2" : "=v"(w.y) : "v"((unsigned int)br), "v"((unsigned int)(bi >> 32)));
    return __builtin_bit_cast(unsigned long long, w);
}

// quant2(a1, b1, a2, b2) rounds a1 b1 + a2 b2 (two points' contributions to one cell).
__device__ inline unsigned long long qbits2(double a1, double b1, double a2, double b2)
{
    return (unsigned long long)__double_as_longlong(fma(a2, b2, fma(a1, b1, QMAGIC)));
}
template <bool FQ> struct SpreadAcc<float, FQ> {
    using U = unsigned int;
    using S = int;
    static constexpr double RANGE = 0x1p31;
    __device__ static U quant(double a, double b) { return (U)qbits(a, b); }
    __device__ static U quant2(double a1, double b1, double a2, double b2)
    {
        return (U)qbits2(a1, b1, a2, b2);
    }
    __device__ static S total(U t) { return (S)t; }
};
template <> struct SpreadAcc<double, false> {
    using U = unsigned long long;
    using S = long long;
    static constexpr double RANGE = 0x1p63;
    __device__ static U quant(double a, double b) { return (U)__double2ll_rn(a * b); }
    __device__ static U quant2(double a1, double b1, double a2, double b2)
    {
        return (U)__double2ll_rn(fma(a2, b2, a1 * b1));
    }
    __device__ static S total(U t) { return (S)t; }
};
template <> struct SpreadAcc<double, true> {
    using U = unsigned long long;
    using S = long long;
    static constexpr double RANGE = 0x1p50;
    __device__ static U quant(double a, double b) { return qbits(a, b); }
    __device__ static U quant2(double a1, double b1, double a2, double b2)
    {
        return qbits2(a1, b1, a2, b2);
    }
    __device__ static S total(U t) { return (S)(t << 13) >> 13; }
};

// Type-1 spreading of one chunk.  The chunk's patch accumulates in fixed point: every
// contribution y w_i w_j is scaled by RANGE (1 - 2^-20) / S with S = sum over the
// chunk's points of |Re y| + |Im y|, which bounds every cell sum, so the
// two's-complement integer adds never wrap; the quantisation step is S / RANGE
// (2^-31 S for FP32, 2^-63 or 2^-50 S for FP64, see SpreadAcc).  Couples of
// neighbouring points go as one window (SPREAD_GAP), the rest one by one; the lanes
// of one atomic instruction visit the couples, then the single points, st apart (see
// spread_stride).  FP32 complex
// grids keep both parts of a cell in one 64-bit word, Re 2^32 + Im (as integers):
// integer addition is exact and associative, and each part's sum stays within
// 32-bit range, so the word's low 32 bits (read as signed) are the sum of the
// imaginary parts and the rest, shifted down, that of the real parts -- one atomic
// per tap and cell instead of two, with the same sums.  FP64 keeps the parts in
// separate planes (row stride g.ps cells).  The points' values are read once (they
// give S and are then spread from LDS).  Non-zero cells are then added to the
// grid: with global atomics (ATOMIC), or with plain read-add-write when no other
// workgroup can touch the patch at the same time (tiles launched by colour).

// Visit order of a chunk's points: slot k takes point (k st) mod n with st the first
// odd number from SPREAD_STRIDE on that is coprime to n (a permutation of the chunk).
// Points next to each other in sorted (cell) order often share a cell, and lanes of
// one atomic instruction on the same address are serialised; lanes st points apart
// rarely share a cell.
constexpr int SPREAD_STRIDE = 97;
__device__ inline int spread_stride(int n)
{
    for (int st = SPREAD_STRIDE;; st += 2) {
        int a = st, b = n;
        while (b) {
            const int t = a % b;
            a = b;
            b = t;
        }
        if (a == 1)
            return st;
    }
}

template <typename T, bool CPLX> struct SpreadPack {
    static constexpr bool value = CPLX && std::is_same<T, float>::value;
};

// Points of a chunk in cell order are mostly one or two cells apart along a row.
// Couples of neighbouring sorted points whose first kernel cells share the row and lie
// at most SPREAD_GAP columns apart (chosen greedily along each run of such
// neighbours) are spread as one window of W rows by W + gap columns (each cell takes
// both contributions in one atomic word); the other points are spread one by one.
constexpr int SPREAD_GAP = 2;

// Waves per SIMD the spreading kernels are compiled for: a 128-register budget
// (FP64 w = 15 needs 135 registers without it; four waves per SIMD instead of three
// took its spreading from 7.24 to 6.41 ms at the benchmark).
constexpr int SPREAD_WAVES = 4;

// Per-chunk staging of the spreading (static LDS beside the patch).
struct SpreadStage {
    short pairs[NUFFT_THREADS];            // couples spread as one window
    short singles[CHUNK];                  // points spread on their own
    int cnt[2 * (NUFFT_THREADS / 64)];     // per wave: couples, single points
    double wsum[NUFFT_THREADS / 64];       // per wave: partial bound S
};
static_assert(sizeof(SpreadStage) <= SPREAD_STAGE_BYTES, "spreading stage within its LDS budget");

// One point per lane at a time: the points' values are read once (they give S and
// are then spread from registers); the lanes of one atomic instruction visit the
// chunk's points st apart in sorted order.  Returns false (nothing spread) when the
// chunk's values are all zero or not finite.
template <typename T, int W, bool CPLX, bool FQ>
__device__ inline bool spread_single(int4 ck, const double *__restrict__ sth,
                                     const double *__restrict__ sph,
                                     const int32_t *__restrict__ perm, const T *__restrict__ in,
                                     const GridGeom &g, T beta, typename SpreadAcc<T, FQ>::U *patch,
                                     double *wsum, int row0, int col0, double &scale)
{
    using A = SpreadAcc<T, FQ>;
    using U = typename A::U;
    constexpr bool PACK = SpreadPack<T, CPLX>::value;
    constexpr int PER = CHUNK / NUFFT_THREADS;
    const int PR = g.t1 + W - 1;
    const int plane = PR * g.ps;
    const int n = ck.z - ck.y;
    // the chunk's values (read once) and the bound S of every cell sum
    const int st = n > 1 ? spread_stride(n) : 1;
    double yr[PER], yi[PER];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int k = threadIdx.x + q * NUFFT_THREADS;
        yr[q] = yi[q] = 0.0;
        if (k < n) {
            const int32_t src = perm[ck.y + (int)(((int64_t)k * st) % n)];
            yr[q] = (double)in[src];
            if constexpr (CPLX)
                yi[q] = (double)in[g.npts + src];
            s += fabs(yr[q]) + fabs(yi[q]);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0)
        wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    double S = 0.0;
#pragma unroll
    for (int w = 0; w < NUFFT_THREADS / 64; ++w)
        S += wsum[w];
    __syncthreads();  // wsum is reused by the next chunk of the same workgroup
    if (!(S > 0.0) || !isfinite(S))
        return false;  // nothing (finite) to spread; uniform over the block
    scale = A::RANGE * (1.0 - 0x1p-20) / S;
    // one rolled loop (a copy of the tap loops per point would double the code)
#pragma unroll 1
    for (int q = 0; q < PER; ++q) {
        const int k = threadIdx.x + q * NUFFT_THREADS;
        if (k >= n)
            break;
        const int p = ck.y + (int)(((int64_t)k * st) % n);
        T wx[W], wy[W];
        int lr, lc;
        point_weights<T, W>(sth[p], sph[p], g, row0, col0, beta, lr, lc, wx, wy);
        if (lr < 0 || lr >= g.t1 || lc < 0 || lc >= g.t2)
            continue;  // cannot happen for points sorted by the same arithmetic
        const double vr = yr[q] * scale, vi = yi[q] * scale;
        double dy[W];
#pragma unroll
        for (int j = 0; j < W; ++j)
            dy[j] = (double)wy[j];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const double fr = (double)wx[i] * vr, fi = (double)wx[i] * vi;
            if constexpr (PACK) {
                unsigned long long *rowp =
                    reinterpret_cast<unsigned long long *>(patch) + (lr + i) * g.ps + lc;
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    // Re 2^32 + Im: the low word is round(Im); the high word takes
                    // round(Re) plus the sign extension of round(Im), which is the
                    // high word of its magic-rounded bits minus KMhi = KM / 2^32
                    // (rounding Re with the constant M - 2^32 KMhi leaves the
                    // subtraction in its low word)
                    const unsigned long long br = (unsigned long long)__double_as_longlong(
                        fma(fr, dy[j], QMAGIC - (double)QMAGIC_HI));
                    const unsigned long long bi = qbits(fi, dy[j]);
                    atomicAdd(rowp + j, pack_word(br, bi));
                }
            } else {
                U *rowp = patch + (lr + i) * g.ps + lc;
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    atomicAdd(rowp + j, A::quant(fr, dy[j]));
                    if constexpr (CPLX)
                        atomicAdd(rowp + plane + j, A::quant(fi, dy[j]));
                }
            }
        }
    }
    return true;
}

// Couples as one window, then the single points (values re-read from the map:
// the preamble's reads leave them in the caches).  Returns false (nothing spread)
// when the chunk's values are all zero or not finite.  OWN_S: the chunk's own bound S
// sets scale; otherwise the caller's scale (a bound over more points) is used.
template <typename T, int W, bool CPLX, bool FQ, bool OWN_S = true>
__device__ inline bool spread_paired(int4 ck, const double *__restrict__ sth,
                                     const double *__restrict__ sph,
                                     const int32_t *__restrict__ perm, const T *__restrict__ in,
                                     const GridGeom &g, T beta, typename SpreadAcc<T, FQ>::U *patch,
                                     SpreadStage &sg, int row0, int col0, double &scale)
{
    using A = SpreadAcc<T, FQ>;
    using U = typename A::U;
    constexpr bool PACK = SpreadPack<T, CPLX>::value;
    constexpr int NW = NUFFT_THREADS / 64;
    constexpr int WG = W + SPREAD_GAP;
    static_assert(2 * NUFFT_THREADS == CHUNK, "two points per thread");
    const int PR = g.t1 + W - 1;
    const int plane = PR * g.ps;  // FP64 complex: real parts, then imaginary parts
    const int n = ck.z - ck.y;
    // Thread t looks at the chunk's points k = t + 256 h (h = 0, 1): wave wv holds the
    // two 64-point segments starting at 64 wv and 256 + 64 wv.  Point k couples with
    // k + 1 when both exist and their first kernel cells share the row at most
    // SPREAD_GAP columns apart (within a segment).  Couples are chosen greedily along
    // each run of such neighbours (its 1st and 2nd point, 3rd and 4th, ...); the
    // other points go one by one.  Also the bound S of every cell sum.
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    bool has[2], start[2], single[2];
    double s = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = t + NUFFT_THREADS * h;
        has[h] = k < n;
        int lr = 0, lc = 0;
        if (has[h]) {
            if constexpr (OWN_S) {
                const int32_t src = perm[ck.y + k];
                const double a = (double)in[src];
                const double b = CPLX ? (double)in[g.npts + src] : 0.0;
                s += fabs(a) + fabs(b);
            }
            const Cell c = point_cell(sth[ck.y + k], sph[ck.y + k], g.c1, g.c2, g.half, g.a_min,
                                      g.n2, g.nrows, W);
            lr = c.r0 - row0;
            lc = c.bi - col0;
        }
        const int lrn = __shfl_down(lr, 1, 64), lcn = __shfl_down(lc, 1, 64);
        const bool hasn = lane < 63 && k + 1 < n;
        const bool cond = has[h] && hasn && lrn == lr && lcn >= lc && lcn - lc <= SPREAD_GAP;
        const unsigned long long cm = __ballot(cond);
        // ones of cm right below this lane: lane - (highest zero below it) - 1
        const unsigned long long zb = ~cm & below;
        const int p0 = zb ? 63 - __clzll((long long)zb) : -1;
        start[h] = cond && ((lane - p0 - 1) & 1) == 0;
        const unsigned long long sm = __ballot(start[h]);
        const bool second = lane > 0 && ((sm >> (lane - 1)) & 1ull);
        single[h] = has[h] && !start[h] && !second;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        s += __shfl_xor(s, d, 64);
    const unsigned long long bp0 = __ballot(start[0]), bp1 = __ballot(start[1]);
    const unsigned long long bs0 = __ballot(single[0]), bs1 = __ballot(single[1]);
    if (lane == 0) {
        if constexpr (OWN_S)  // (otherwise the caller may still be reading wsum)
            sg.wsum[wv] = s;
        sg.cnt[wv] = __popcll(bp0) + __popcll(bp1);
        sg.cnt[NW + wv] = __popcll(bs0) + __popcll(bs1);
    }
    __syncthreads();
    double S = 0.0;
    int npair = 0, nsing = 0, opair = 0, osing = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if constexpr (OWN_S)
            S += sg.wsum[w];
        const int cp = sg.cnt[w], cs = sg.cnt[NW + w];
        if (w < wv) {
            opair += cp;
            osing += cs;
        }
        npair += cp;
        nsing += cs;
    }
    // couples by their first point, then the single points (segment 0, then 1)
    if (start[0])
        sg.pairs[opair + __popcll(bp0 & below)] = (short)t;
    if (start[1])
        sg.pairs[opair + __popcll(bp0) + __popcll(bp1 & below)] = (short)(t + NUFFT_THREADS);
    if (single[0])
        sg.singles[osing + __popcll(bs0 & below)] = (short)t;
    if (single[1])
        sg.singles[osing + __popcll(bs0) + __popcll(bs1 & below)] = (short)(t + NUFFT_THREADS);
    __syncthreads();
    if constexpr (OWN_S) {
        if (!(S > 0.0) || !isfinite(S))
            return false;  // nothing (finite) to spread; uniform over the block
        scale = A::RANGE * (1.0 - 0x1p-20) / S;
    }
    auto value = [&](int p, double &vr, double &vi) {
        const int32_t src = perm[p];
        vr = (double)in[src] * scale;
        vi = CPLX ? (double)in[g.npts + src] * scale : 0.0;
    };
    // windows of couples (at most one per thread), visited st apart
    {
        const int st = npair > 1 ? spread_stride(npair) : 1;
        const int i = t;
        if (i < npair) {
            const int k = sg.pairs[(int)(((int64_t)i * st) % npair)];
            const int pa = ck.y + k;
            T wxa[W], wya[W], wxb[W], wyb[W];
            int lra, lca, lrb, lcb;
            point_weights<T, W>(sth[pa], sph[pa], g, row0, col0, beta, lra, lca, wxa, wya);
            point_weights<T, W>(sth[pa + 1], sph[pa + 1], g, row0, col0, beta, lrb, lcb, wxb, wyb);
            const int gap = lcb - lca;  // 0..SPREAD_GAP, same row (checked above)
            if (lra >= 0 && lra < g.t1 && lca >= 0 && lcb < g.t2) {
                // column weights over the window: a's at 0..W-1, b's shifted by gap
                double da[WG], db[WG];
#pragma unroll
                for (int j = 0; j < WG; ++j) {
                    da[j] = j < W ? (double)wya[j] : 0.0;
                    double v = 0.0;
#pragma unroll
                    for (int gg = 0; gg <= SPREAD_GAP; ++gg)
                        if (j - gg >= 0 && j - gg < W && gap == gg)
                            v = (double)wyb[j - gg];
                    db[j] = v;
                }
                double vra, via, vrb, vib;
                value(pa, vra, via);
                value(pa + 1, vrb, vib);
#pragma unroll
                for (int i2 = 0; i2 < W; ++i2) {
                    const double fra = (double)wxa[i2] * vra, fia = (double)wxa[i2] * via;
                    const double frb = (double)wxb[i2] * vrb, fib = (double)wxb[i2] * vib;
                    // cell (lra + i2, lca) of the patch: 64-bit words when packed
                    const int cell0 = (lra + i2) * g.ps + lca;
                    U *rowp = patch + cell0;
                    unsigned long long *roww = reinterpret_cast<unsigned long long *>(patch) + cell0;
#pragma unroll
                    for (int j = 0; j < WG; ++j) {
                        if (j >= W && j >= W + gap)
                            continue;  // beyond b's window
                        if constexpr (PACK) {
                            const unsigned long long br = (unsigned long long)__double_as_longlong(
                                fma(frb, db[j], fma(fra, da[j], QMAGIC - (double)QMAGIC_HI)));
                            const unsigned long long bi = (unsigned long long)__double_as_longlong(
                                fma(fib, db[j], fma(fia, da[j], QMAGIC)));
                            atomicAdd(roww + j, pack_word(br, bi));
                        } else {
                            atomicAdd(rowp + j, A::quant2(fra, da[j], frb, db[j]));
                            if constexpr (CPLX)
                                atomicAdd(rowp + plane + j, A::quant2(fia, da[j], fib, db[j]));
                        }
                    }
                }
            }
        }
    }
    // the other points one by one (one rolled loop: a copy of the tap loops per
    // point would double the code)
    const int st = nsing > 1 ? spread_stride(nsing) : 1;
#pragma unroll 1
    for (int i = t; i < nsing; i += NUFFT_THREADS) {
        const int k = sg.singles[(int)(((int64_t)i * st) % nsing)];
        const int p = ck.y + k;
        T wx[W], wy[W];
        int lr, lc;
        point_weights<T, W>(sth[p], sph[p], g, row0, col0, beta, lr, lc, wx, wy);
        if (lr < 0 || lr >= g.t1 || lc < 0 || lc >= g.t2)
            continue;  // cannot happen for points sorted by the same arithmetic
        double vr, vi;
        value(p, vr, vi);
        double dy[W];
#pragma unroll
        for (int j = 0; j < W; ++j)
            dy[j] = (double)wy[j];
#pragma unroll
        for (int i2 = 0; i2 < W; ++i2) {
            const double fr = (double)wx[i2] * vr, fi = (double)wx[i2] * vi;
            if constexpr (PACK) {
                unsigned long long *rowp =
                    reinterpret_cast<unsigned long long *>(patch) + (lr + i2) * g.ps + lc;
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    // Re 2^32 + Im: the low word is round(Im); the high word takes
                    // round(Re) plus the sign extension of round(Im), which is the
                    // high word of its magic-rounded bits minus KMhi = KM / 2^32
                    // (rounding Re with the constant M - 2^32 KMhi leaves the
                    // subtraction in its low word)
                    const unsigned long long br = (unsigned long long)__double_as_longlong(
                        fma(fr, dy[j], QMAGIC - (double)QMAGIC_HI));
                    const unsigned long long bi = qbits(fi, dy[j]);
                    atomicAdd(rowp + j, pack_word(br, bi));
                }
            } else {
                U *rowp = patch + (lr + i2) * g.ps + lc;
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    atomicAdd(rowp + j, A::quant(fr, dy[j]));
                    if constexpr (CPLX)
                        atomicAdd(rowp + plane + j, A::quant(fi, dy[j]));
                }
            }
        }
    }
    return true;
}

// Adds a spread patch (fixed point, step 1 / scale) to the grid: with global atomics
// (ATOMIC), or with plain read-add-write when no other workgroup can touch the patch
// at the same time (tiles launched by colour).  The caller has synchronised the block.
template <typename T, int W, bool CPLX, bool ATOMIC, bool FQ>
__device__ inline void flush_patch(const typename SpreadAcc<T, FQ>::U *patch, const GridGeom &g,
                                   int row0, int col0, double scale, T *__restrict__ grid)
{
    using A = SpreadAcc<T, FQ>;
    constexpr bool PACK = SpreadPack<T, CPLX>::value;
    constexpr int NC = CPLX ? 2 : 1;
    const int PR = g.t1 + W - 1, PC = g.t2 + W - 1;
    const int plane = PR * g.ps;  // FP64 complex: real parts, then imaginary parts
    const double inv = 1.0 / scale;
    for (int idx = threadIdx.x; idx < PR * PC; idx += NUFFT_THREADS) {
        const int pr = idx / PC, pc = idx - (idx / PC) * PC;
        const int r = row0 + pr;
        if (r >= g.nrows)
            continue;
        int c = col0 + pc;
        while (c >= g.n2)  // patches may span the torus more than once when n2 is small
            c -= g.n2;
        T *dst = grid + ((size_t)r * g.stride + c) * NC;
        const int pidx = pr * g.ps + pc;
        typename A::S qr, qi;
        if constexpr (PACK) {
            const long long t = (long long)reinterpret_cast<const unsigned long long *>(patch)[pidx];
            qi = (int)(unsigned int)(t & 0xffffffffll);
            qr = (int)((t - (long long)qi) >> 32);
        } else {
            qr = A::total(patch[pidx]);
            qi = CPLX ? A::total(patch[plane + pidx]) : 0;
        }
        if (ATOMIC) {
            if (qr != 0)
                unsafeAtomicAdd(dst, (T)((double)qr * inv));
            if (CPLX && qi != 0)
                unsafeAtomicAdd(dst + 1, (T)((double)qi * inv));
        } else if (qr != 0 || qi != 0) {
            if constexpr (CPLX) {
                using C2 = typename cpl<T>::type;
                C2 v = *reinterpret_cast<C2 *>(dst);
                v.x += (T)((double)qr * inv);
                v.y += (T)((double)qi * inv);
                *reinterpret_cast<C2 *>(dst) = v;
            } else {
                *dst += (T)((double)qr * inv);
            }
        }
    }
}

// Spreading of one chunk into its patch, then the flush of the patch to the grid.
// FP64 grids spread couples of neighbouring points as one window (fewer LDS
// atomics, which bound them); FP32 grids, bound by their arithmetic, point by point.
template <typename T, int W, bool CPLX, bool ATOMIC, bool FQ>
__device__ inline void spread_chunk(int4 ck, const double *__restrict__ sth,
                                    const double *__restrict__ sph,
                                    const int32_t *__restrict__ perm, const T *__restrict__ in,
                                    const GridGeom &g, T beta, T *__restrict__ grid,
                                    typename SpreadAcc<T, FQ>::U *patch, SpreadStage &sg)
{
    constexpr int NC = CPLX ? 2 : 1;
    const int tr = ck.x / g.nt2, tc = ck.x - (ck.x / g.nt2) * g.nt2;
    const int row0 = tr * g.t1, col0 = tc * g.t2;
    const int PR = g.t1 + W - 1;
    for (int idx = threadIdx.x; idx < PR * g.ps * NC; idx += NUFFT_THREADS)
        patch[idx] = 0;
    double scale = 0.0;
    bool any;
    if constexpr (std::is_same<T, double>::value)
        any = spread_paired<T, W, CPLX, FQ>(ck, sth, sph, perm, in, g, beta, patch, sg, row0, col0,
                                            scale);
    else
        any = spread_single<T, W, CPLX, FQ>(ck, sth, sph, perm, in, g, beta, patch, sg.wsum, row0,
                                            col0, scale);
    if (!any)
        return;
    __syncthreads();
    flush_patch<T, W, CPLX, ATOMIC, FQ>(patch, g, row0, col0, scale, grid);
    __syncthreads();  // the patch is reused by the next chunk of the same workgroup
}

// FP64 tiles of at most SPREAD_TILE_CHUNKS chunks are spread as a whole into one patch
// (cleared and flushed once) with one bound S over the tile's points: at most two
// chunks' worth, so the quantisation step S / RANGE stays within twice the per-chunk
// one (2^-50 S of at most 1024 values in the fast form, far below the epsilon it
// serves).  Denser tiles go chunk by chunk.
constexpr int SPREAD_TILE_CHUNKS = 2;

// FP64, a whole tile (chunks first .. first + count - 1, one contiguous range of
// points) into one patch, plain read-add-write (tiles launched by colour).
template <int W, bool CPLX, bool FQ>
__device__ inline void spread_tile_f64(int2 it, const int4 *__restrict__ chunks,
                                       const double *__restrict__ sth,
                                       const double *__restrict__ sph,
                                       const int32_t *__restrict__ perm,
                                       const double *__restrict__ in, const GridGeom &g,
                                       double beta, double *__restrict__ grid,
                                       typename SpreadAcc<double, FQ>::U *patch, SpreadStage &sg)
{
    using A = SpreadAcc<double, FQ>;
    constexpr int NC = CPLX ? 2 : 1;
    constexpr int NW = NUFFT_THREADS / 64;
    const int4 c0 = chunks[it.x];
    const int y0 = c0.y, z1 = chunks[it.x + it.y - 1].z;
    const int tr = c0.x / g.nt2, tc = c0.x - (c0.x / g.nt2) * g.nt2;
    const int row0 = tr * g.t1, col0 = tc * g.t2;
    const int PR = g.t1 + W - 1;
    double s = 0.0;
    for (int p = y0 + (int)threadIdx.x; p < z1; p += NUFFT_THREADS) {
        const int32_t src = perm[p];
        s += fabs(in[src]) + (CPLX ? fabs(in[g.npts + src]) : 0.0);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0)
        sg.wsum[threadIdx.x >> 6] = s;
    for (int idx = threadIdx.x; idx < PR * g.ps * NC; idx += NUFFT_THREADS)
        patch[idx] = 0;
    __syncthreads();
    double S = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w)
        S += sg.wsum[w];
    if (!(S > 0.0) || !isfinite(S))
        return;  // nothing (finite) to spread; uniform over the block
    double scale = A::RANGE * (1.0 - 0x1p-20) / S;
    for (int c = 0; c < it.y; ++c)
        spread_paired<double, W, CPLX, FQ, false>(chunks[it.x + c], sth, sph, perm, in, g, beta,
                                                  patch, sg, row0, col0, scale);
    __syncthreads();
    flush_patch<double, W, CPLX, false, FQ>(patch, g, row0, col0, scale, grid);
}

// One workgroup per chunk, atomic flush (any grid).
template <typename T, int W, bool CPLX, bool FQ>
__global__ __launch_bounds__(NUFFT_THREADS, SPREAD_WAVES) void spread_kernel(
    const int4 *__restrict__ chunks, const double *__restrict__ sth, const double *__restrict__ sph,
    const int32_t *__restrict__ perm, const T *__restrict__ in, GridGeom g, T beta,
    T *__restrict__ grid)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ SpreadStage sg;
    spread_chunk<T, W, CPLX, true, FQ>(chunks[blockIdx.x], sth, sph, perm, in, g, beta, grid,
                                       reinterpret_cast<typename SpreadAcc<T, FQ>::U *>(smem_raw),
                                       sg);
}

// One workgroup per tile of one colour (all of the tile's chunks in turn), plain
// read-add-write flush: tiles of one colour are at least two tiles apart in both
// directions and a patch reaches only W - 1 cells beyond its tile, so their
// patches are disjoint.  items[i] = (first chunk, number of chunks).
template <typename T, int W, bool CPLX, bool FQ>
__global__ __launch_bounds__(NUFFT_THREADS, SPREAD_WAVES) void spread_tile_kernel(
    const int2 *__restrict__ items, const int4 *__restrict__ chunks,
    const double *__restrict__ sth, const double *__restrict__ sph,
    const int32_t *__restrict__ perm, const T *__restrict__ in, GridGeom g, T beta,
    T *__restrict__ grid)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ SpreadStage sg;
    const int2 it = items[blockIdx.x];
    auto *patch = reinterpret_cast<typename SpreadAcc<T, FQ>::U *>(smem_raw);
    if (std::is_same<T, double>::value && it.y <= SPREAD_TILE_CHUNKS) {
        if constexpr (std::is_same<T, double>::value)
            spread_tile_f64<W, CPLX, FQ>(it, chunks, sth, sph, perm, in, g, beta, grid, patch, sg);
    } else {
        for (int c = 0; c < it.y; ++c)
            spread_chunk<T, W, CPLX, false, FQ>(chunks[it.x + c], sth, sph, perm, in, g, beta,
                                                grid, patch, sg);
    }
}

static GridGeom make_geom(const gsht_plan &p)
{
    GridGeom g;
    g.c1 = (double)p.n1 / (2.0 * 3.141592653589793);
    g.c2 = (double)p.n2 / (2.0 * 3.141592653589793);
    g.half = 0.5 * (double)p.w;
    g.a_min = p.a_min;
    g.n2 = p.n2;
    g.stride = p.n2;  // complex grid: n2 complex per row; real grid: n2 reals per row
    g.nrows = p.nrows;
    g.t1 = p.t1;
    g.t2 = p.t2;
    g.nt2 = p.nt2;
    g.ps = p.t2 + p.w - 1;
    g.npts = p.npts;
    g.poly = p.es_poly;
    return g;
}

template <typename T, int W>
static hipError_t interp_w(const gsht_plan &p, void *map, hipStream_t s)
{
    const GridGeom g = make_geom(p);
    const int PR = p.t1 + W - 1, PS = p.t2 + W - 1;
    // FP64: one workgroup per tile when the tile list exists (built with the spreading
    // colours), so each 32 KB patch is loaded once (w = 14: 2.98 -> 2.78 ms at the
    // benchmark); FP32 patches are small and the chunks balance better (0.83 -> 0.84 ms
    // per tile), so FP32 stays per chunk
    const int2 *items =
        (std::is_same<T, double>::value && p.ncolors > 0) ? p.tile_items : nullptr;
    const unsigned nb = (unsigned)(items ? p.color_start[p.ncolors] : p.nchunks);
    if (p.spin) {
        const size_t sm = (size_t)PR * PS * sizeof(typename cpl<T>::type);
        hipLaunchKernelGGL((interp_kernel<T, W, true>), dim3(nb), dim3(NUFFT_THREADS), sm, s,
                           p.chunks, items, p.sth, p.sph, p.perm, p.G, g, (T)p.beta, (T *)map);
    } else {
        const size_t sm = (size_t)PR * PS * sizeof(T);
        hipLaunchKernelGGL((interp_kernel<T, W, false>), dim3(nb), dim3(NUFFT_THREADS), sm, s,
                           p.chunks, items, p.sth, p.sph, p.perm, p.g, g, (T)p.beta, (T *)map);
    }
    return hipGetLastError();
}

struct DerivOut {
    void *map, *dth, *dph;
    const void *gin;
    double *gth, *gph;
};

template <typename T, int W>
static hipError_t interp_deriv_w(const gsht_plan &p, const DerivOut &o, hipStream_t s)
{
    const GridGeom g = make_geom(p);
    const int PR = p.t1 + W - 1, PS = p.t2 + W - 1;
    const bool vjp = o.gin != nullptr;
    const dim3 grd((unsigned)p.nchunks), blk(NUFFT_THREADS);
    T *map = (T *)o.map, *dth = (T *)o.dth, *dph = (T *)o.dph;
    const T *gin = (const T *)o.gin;
    if (p.spin) {
        const size_t sm = (size_t)PR * PS * sizeof(typename cpl<T>::type);
        if (vjp)
            hipLaunchKernelGGL((interp_deriv_kernel<T, W, true, true>), grd, blk, sm, s, p.chunks,
                               p.sth, p.sph, p.perm, p.G, g, (T)p.beta, map, dth, dph, gin, o.gth,
                               o.gph);
        else
            hipLaunchKernelGGL((interp_deriv_kernel<T, W, true, false>), grd, blk, sm, s, p.chunks,
                               p.sth, p.sph, p.perm, p.G, g, (T)p.beta, map, dth, dph, gin, o.gth,
                               o.gph);
    } else {
        const size_t sm = (size_t)PR * PS * sizeof(T);
        if (vjp)
            hipLaunchKernelGGL((interp_deriv_kernel<T, W, false, true>), grd, blk, sm, s, p.chunks,
                               p.sth, p.sph, p.perm, p.g, g, (T)p.beta, map, dth, dph, gin, o.gth,
                               o.gph);
        else
            hipLaunchKernelGGL((interp_deriv_kernel<T, W, false, false>), grd, blk, sm, s,
                               p.chunks, p.sth, p.sph, p.perm, p.g, g, (T)p.beta, map, dth, dph,
                               gin, o.gth, o.gph);
    }
    return hipGetLastError();
}

template <typename T, int W, bool FQ>
static hipError_t spread_wq(const gsht_plan &p, const void *map, hipStream_t s)
{
    const GridGeom g = make_geom(p);
    const int PR = p.t1 + W - 1, PS = p.t2 + W - 1;
    using U = typename SpreadAcc<T, FQ>::U;
    if (p.ncolors > 0) {
        const size_t sm = (size_t)PR * PS * (p.spin ? 2 : 1) * sizeof(U);
        for (int c = 0; c < p.ncolors; ++c) {
            const int n = p.color_start[c + 1] - p.color_start[c];
            if (n == 0)
                continue;
            const int2 *items = p.tile_items + p.color_start[c];
            if (p.spin)
                hipLaunchKernelGGL((spread_tile_kernel<T, W, true, FQ>), dim3((unsigned)n),
                                   dim3(NUFFT_THREADS), sm, s, items, p.chunks, p.sth, p.sph,
                                   p.perm, (const T *)map, g, (T)p.beta, (T *)p.G);
            else
                hipLaunchKernelGGL((spread_tile_kernel<T, W, false, FQ>), dim3((unsigned)n),
                                   dim3(NUFFT_THREADS), sm, s, items, p.chunks, p.sth, p.sph,
                                   p.perm, (const T *)map, g, (T)p.beta, (T *)p.g);
        }
        return hipGetLastError();
    }
    if (p.spin) {
        const size_t sm = (size_t)PR * PS * 2 * sizeof(U);
        hipLaunchKernelGGL((spread_kernel<T, W, true, FQ>), dim3((unsigned)p.nchunks),
                           dim3(NUFFT_THREADS), sm, s, p.chunks, p.sth, p.sph, p.perm,
                           (const T *)map, g, (T)p.beta, (T *)p.G);
    } else {
        const size_t sm = (size_t)PR * PS * sizeof(U);
        hipLaunchKernelGGL((spread_kernel<T, W, false, FQ>), dim3((unsigned)p.nchunks),
                           dim3(NUFFT_THREADS), sm, s, p.chunks, p.sth, p.sph, p.perm,
                           (const T *)map, g, (T)p.beta, (T *)p.g);
    }
    return hipGetLastError();
}

// FP32 grids always take the magic rounding; FP64 grids take it where the plan's
// accuracy allows (gsht_plan::spread_fast).
template <typename T, int W>
static hipError_t spread_w(const gsht_plan &p, const void *map, hipStream_t s)
{
    if constexpr (sizeof(T) == 8) {
        if (!p.spread_fast)
            return spread_wq<T, W, false>(p, map, s);
    }
    return spread_wq<T, W, true>(p, map, s);
}

#define GSHT_W_CASES(F, T)                                                                       \
    switch (p.w) {                                                                               \
    case 4: return F<T, 4>(p, map, s);                                                           \
    case 5: return F<T, 5>(p, map, s);                                                           \
    case 6: return F<T, 6>(p, map, s);                                                           \
    case 7: return F<T, 7>(p, map, s);                                                           \
    case 8: return F<T, 8>(p, map, s);                                                           \
    case 9: return F<T, 9>(p, map, s);                                                           \
    case 10: return F<T, 10>(p, map, s);                                                         \
    case 11: return F<T, 11>(p, map, s);                                                         \
    case 12: return F<T, 12>(p, map, s);                                                         \
    case 13: return F<T, 13>(p, map, s);                                                         \
    case 14: return F<T, 14>(p, map, s);                                                         \
    case 15: return F<T, 15>(p, map, s);                                                         \
    case 16: return F<T, 16>(p, map, s);                                                         \
    default: return hipErrorInvalidValue;                                                        \
    }

#define GSHT_W_CASES_F32(F)                                                                      \
    switch (p.w) {                                                                               \
    case 4: return F<float, 4>(p, map, s);                                                       \
    case 5: return F<float, 5>(p, map, s);                                                       \
    case 6: return F<float, 6>(p, map, s);                                                       \
    case 7: return F<float, 7>(p, map, s);                                                       \
    case 8: return F<float, 8>(p, map, s);                                                       \
    default: return hipErrorInvalidValue;                                                        \
    }

hipError_t launch_interp(const gsht_plan &p, void *map, hipStream_t s)
{
    if (p.nchunks == 0)
        return hipSuccess;
    if (p.prec == GSHT_F64) {
        GSHT_W_CASES(interp_w, double)
    } else {
        GSHT_W_CASES_F32(interp_w)
    }
}

hipError_t launch_interp_deriv(const gsht_plan &p, void *out_map, void *dth, void *dph,
                              const void *gin, double *gth, double *gph, hipStream_t s)
{
    if (p.nchunks == 0)
        return hipSuccess;
    const DerivOut map{out_map, dth, dph, gin, gth, gph};  // the W switch passes "map" on
    if (p.prec == GSHT_F64) {
        GSHT_W_CASES(interp_deriv_w, double)
    } else {
        GSHT_W_CASES_F32(interp_deriv_w)
    }
}

hipError_t launch_spread(const gsht_plan &p, const void *map, hipStream_t s)
{
    if (p.nchunks == 0)
        return hipSuccess;
    if (p.prec == GSHT_F64) {
        GSHT_W_CASES(spread_w, double)
    } else {
        GSHT_W_CASES_F32(spread_w)
    }
}

}  // namespace gsht

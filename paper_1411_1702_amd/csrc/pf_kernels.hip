// pf_kernels.hip -- the device side of one assimilation step (Algorithm 1,
// steps 2-6) for a batch of filters, plus filter initialisation (step 1).
//
// Work is a list of (batch entry, tile) items; a workgroup of TILE lanes
// owns one tile of TILE particles, one particle per lane.  Kernels loop over
// the list (grid-stride), so one launch covers every filter in the batch.
// Per-filter reductions use fixed tiles combined in a fixed order, so a
// filter's arithmetic never depends on what else is in the batch.  No kernel
// waits on another workgroup: whatever a tile needs from the whole filter
// (the first-stage log-sum-exp, the integer CDF offset of its tile) it
// recomputes from the previous kernel's per-tile partials, in the same fixed
// order in every workgroup.
//
//   k_predict  : shrink, predictor Psi, first-stage log-weights, tile
//                (max, sum exp)                                    steps 2, 3a
//   k_count    : filter log-sum-exp from the tile partials; integer weights
//                q = floor(g 2^S); tile sums                       step 3b
//   k_scatter  : tile offset and total of the integer CDF, systematic
//                offset V, ancestors by scatter                    step 3b
//   k_update   : gather, proliferate, Psi with local-error estimate,
//                innovation, second-stage log-weights, tile moments
//                                                                  steps 3c-5
//   k_moments  : one workgroup per filter: mean, covariance, ESS, Cholesky,
//                commit, status by ticket                          step 6
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pf_device.hpp"
#include "pf_types.hpp"

namespace pf {

constexpr int WAVE = 64;
constexpr int NWAVE = TILE / WAVE;

// ---------------------------------------------------------------------------
// wavefront reductions with DPP lane moves (VALU operand modifiers, no LDS
// round trip): pairs, quads, half rows, rows, then the two row broadcasts of
// wave64.  A fixed tree, so results are deterministic; the full result lands
// in lane 63 and is broadcast with readlane.
// ---------------------------------------------------------------------------
constexpr int DPP_QUAD_1032 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_2301 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_ROW_MIRROR = 0x140;
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_BCAST15 = 0x142;
constexpr int DPP_ROW_BCAST31 = 0x143;

template <int CTRL, int ROWS>
__device__ inline uint64_t dpp64(uint64_t v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xF, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
template <int CTRL, int ROWS>
__device__ inline double dppd(double v)
{
    return __longlong_as_double((long long)dpp64<CTRL, ROWS>((uint64_t)__double_as_longlong(v)));
}
__device__ inline uint64_t lane63_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline double lane63(double v)
{
    return __longlong_as_double((long long)lane63_u64((uint64_t)__double_as_longlong(v)));
}

// orders one wavefront's LDS writes before its lanes' later reads (a
// wavefront's LDS operations complete in order; the fences keep the
// compiler from moving them across this point)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double wave_sum(double v)
{
    v += dppd<DPP_QUAD_1032, 0xF>(v);
    v += dppd<DPP_QUAD_2301, 0xF>(v);
    v += dppd<DPP_ROW_HALF_MIRROR, 0xF>(v);
    v += dppd<DPP_ROW_MIRROR, 0xF>(v);
    v += dppd<DPP_ROW_BCAST15, 0xA>(v);
    v += dppd<DPP_ROW_BCAST31, 0xC>(v);
    return lane63(v);
}
// max: lanes outside the broadcast rows receive 0 from the move, so the
// broadcast steps use the -inf-padded form max(v, move(v) or v)
__device__ inline double wave_max(double v)
{
    v = fmax(v, dppd<DPP_QUAD_1032, 0xF>(v));
    v = fmax(v, dppd<DPP_QUAD_2301, 0xF>(v));
    v = fmax(v, dppd<DPP_ROW_HALF_MIRROR, 0xF>(v));
    v = fmax(v, dppd<DPP_ROW_MIRROR, 0xF>(v));
    const uint32_t row = (__lane_id() >> 4);
    const double b15 = dppd<DPP_ROW_BCAST15, 0xA>(v);
    if (row & 1) v = fmax(v, b15);
    const double b31 = dppd<DPP_ROW_BCAST31, 0xC>(v);
    if (row >= 2) v = fmax(v, b31);
    return lane63(v);
}
__device__ inline unsigned long long wave_sum_u64(unsigned long long v)
{
    v += dpp64<DPP_QUAD_1032, 0xF>(v);
    v += dpp64<DPP_QUAD_2301, 0xF>(v);
    v += dpp64<DPP_ROW_HALF_MIRROR, 0xF>(v);
    v += dpp64<DPP_ROW_MIRROR, 0xF>(v);
    v += dpp64<DPP_ROW_BCAST15, 0xA>(v);
    v += dpp64<DPP_ROW_BCAST31, 0xC>(v);
    return lane63_u64(v);
}

__device__ inline double block_max(double v, double* sh)
{
    v = wave_max(v);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int i = 1; i < NWAVE; ++i) r = fmax(r, sh[i]);
    return r;
}
__device__ inline double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int i = 1; i < NWAVE; ++i) r += sh[i];
    return r;
}
__device__ inline unsigned long long block_sum_u64(unsigned long long v, unsigned long long* sh)
{
    v = wave_sum_u64(v);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    unsigned long long r = sh[0];
#pragma unroll
    for (int i = 1; i < NWAVE; ++i) r += sh[i];
    return r;
}

// two block sums at once (one barrier pair); sh holds 2*NWAVE words
__device__ inline void block_sum2_u64(unsigned long long a, unsigned long long b, unsigned long long* sh,
                                      unsigned long long& sa, unsigned long long& sb)
{
    a = wave_sum_u64(a);
    b = wave_sum_u64(b);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) {
        sh[w] = a;
        sh[NWAVE + w] = b;
    }
    __syncthreads();
    sa = sh[0];
    sb = sh[NWAVE];
#pragma unroll
    for (int i = 1; i < NWAVE; ++i) {
        sa += sh[i];
        sb += sh[NWAVE + i];
    }
}

// inclusive prefix sum over the wavefront (uint64, exact) with DPP lane
// moves: shifts by 1, 2, 4, 8 within each row of 16 (lanes without a source
// add 0), then the row broadcasts of lane 15 and lane 31 into the rows above
constexpr int DPP_ROW_SR1 = 0x111, DPP_ROW_SR2 = 0x112, DPP_ROW_SR4 = 0x114, DPP_ROW_SR8 = 0x118;
__device__ inline unsigned long long wave_incl_scan_u64(unsigned long long v)
{
    v += dpp64<DPP_ROW_SR1, 0xF>(v);
    v += dpp64<DPP_ROW_SR2, 0xF>(v);
    v += dpp64<DPP_ROW_SR4, 0xF>(v);
    v += dpp64<DPP_ROW_SR8, 0xF>(v);
    v += dpp64<DPP_ROW_BCAST15, 0xA>(v);
    v += dpp64<DPP_ROW_BCAST31, 0xC>(v);
    return v;
}

// exclusive prefix sum over the block (uint64, exact); returns the total
__device__ inline unsigned long long block_exscan_u64(unsigned long long v, unsigned long long& excl,
                                                      unsigned long long* sh)
{
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    const unsigned long long incl = wave_incl_scan_u64(v);
    __syncthreads();
    if (l == WAVE - 1) sh[w] = incl;
    __syncthreads();
    unsigned long long base = 0, total = 0;
#pragma unroll
    for (int i = 0; i < NWAVE; ++i) {
        if (i < w) base += sh[i];
        total += sh[i];
    }
    excl = base + incl - v;
    return total;
}

// Newton counters of one lane in one word, so a wavefront adds them with one
// reduction: iterations in bits 0-31, failed solves in bits 32-55,
// non-finite weights in bits 56-63 (a lane makes at most substeps*kmax <=
// 2^22 iterations and substeps <= 2^16 failures, so 64 lanes fit).
__device__ inline uint64_t pack_counts(uint32_t iters, uint32_t fails, uint32_t nonf)
{
    return (uint64_t)iters | ((uint64_t)fails << 32) | ((uint64_t)nonf << 56);
}
__device__ inline double count_iters(uint64_t w) { return (double)(w & 0xFFFFFFFFull); }
__device__ inline double count_fails(uint64_t w) { return (double)((w >> 32) & 0xFFFFFFull); }
__device__ inline double count_nonf(uint64_t w) { return (double)(w >> 56); }

// The same combination in one pass for a few columns (small models; the
// first-stage partials): each lane visits its tiles (round-robin, two in
// flight) in increasing order with the NS sums in registers, relative to its
// own running max; then the block max, one rescale per lane, and a block sum
// per column.
template <int NS>
__device__ __forceinline__ double combine_rows(const double* part, int cs, int ntiles, int sq, int nplain, double* out,
                                               double* sh)
{
    constexpr int NA = NS + 1;
    __shared__ double colsum[NWAVE][NS];
    double acc[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] = 0.0;
    double mloc = -INFINITY;
    auto scale = [&](int a, double r) { return a >= NS - nplain ? 1.0 : a == sq ? r * r : r; };
    auto take = [&](const double (&row)[NA]) {
        const double mt = row[0];
        if (mt > mloc) {
            const double r = mloc > -INFINITY ? exp(mloc - mt) : 0.0;
#pragma unroll
            for (int a = 0; a < NS; ++a) acc[a] *= scale(a, r);
            mloc = mt;
        }
        const double sc = mt > -INFINITY ? exp(mt - mloc) : 0.0;
#pragma unroll
        for (int a = 0; a < NS; ++a) acc[a] += scale(a, sc) * row[1 + a];
    };
    for (int t = threadIdx.x; t < ntiles; t += 2 * TILE) {
        const int t2 = t + TILE;
        double r0[NA], r1[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) r0[k] = part[(size_t)k * cs + t];
        if (t2 < ntiles) {
#pragma unroll
            for (int k = 0; k < NA; ++k) r1[k] = part[(size_t)k * cs + t2];
        }
        take(r0);
        if (t2 < ntiles) take(r1);
    }
    const double M = block_max(mloc, sh);
    const double r = (mloc > -INFINITY && M > -INFINITY) ? exp(mloc - M) : 0.0;
    const int w = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
#pragma unroll
    for (int a = 0; a < NS; ++a) {
        const double v = wave_sum(acc[a] * scale(a, r));
        if (ln == 0) colsum[w][a] = v;
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NWAVE; ++i) s += colsum[i][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
    return M;
}

// ---------------------------------------------------------------------------
// Sixteen sums over a row of 16 lanes at once.  Four butterfly levels pair
// lanes that differ in bit 3, 2, 1, 0 of the lane index (DPP row_mirror,
// row_half_mirror, quad_perm [3,2,1,0], quad_perm [1,0,3,2]; each pairing
// keeps the lower bits' partners in the same half).  At each level a lane
// keeps half of its values (the upper half when its bit is set), adds the
// partner's copy of that half and hands over the other half.  Afterwards
// lane l holds value l % 16 summed over its row: 105 VALU operations for
// what sixteen separate reductions do in ~300.
// ---------------------------------------------------------------------------
constexpr int DPP_QUAD_3210 = 0x1B;      // quad_perm [3,2,1,0]

template <int CTRL, int H>
__device__ __forceinline__ void butterfly(double (&v)[16], bool upper)
{
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double keep = upper ? v[i + H] : v[i];
        const double give = upper ? v[i] : v[i + H];
        v[i] = keep + dppd<CTRL, 0xF>(give);
    }
}
__device__ __forceinline__ double row_sum16(double (&v)[16])
{
    const int ln = (int)__lane_id();
    butterfly<DPP_ROW_MIRROR, 8>(v, ln & 8);
    butterfly<DPP_ROW_HALF_MIRROR, 4>(v, ln & 4);
    butterfly<DPP_QUAD_3210, 2>(v, ln & 2);
    butterfly<DPP_QUAD_1032, 1>(v, ln & 1);
    return v[0];
}

// The combination for at most TILE tiles and many columns (the chain's
// moments): one tile per lane, all its columns loaded at once (coalesced
// across lanes, one memory round trip), the block max of the tile maxima,
// each lane scales its own values, and the columns are summed sixteen at a
// time with row_sum16, then across rows and wavefronts in LDS.
template <int NS>
__device__ __forceinline__ double combine_wide(const double* part, int cs, int ntiles, int sq, int nplain,
                                               double* out, double* sh)
{
    constexpr int NCH = (NS + 15) / 16;
    __shared__ double csum[NWAVE][NCH][WAVE];
    const int t = threadIdx.x;
    double v[NCH * 16];
    double mt = -INFINITY;
    if (t < ntiles) {
        mt = part[t];
#pragma unroll
        for (int a = 0; a < NS; ++a) v[a] = part[(size_t)(1 + a) * cs + t];
    } else {
#pragma unroll
        for (int a = 0; a < NS; ++a) v[a] = 0.0;
    }
#pragma unroll
    for (int a = NS; a < NCH * 16; ++a) v[a] = 0.0;
    const double M = block_max(mt, sh);
    const double sc = (mt > -INFINITY && M > -INFINITY) ? exp(mt - M) : 0.0;
    const int w = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        double chunk[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int a = 16 * c + k;
            chunk[k] = v[a] * (a >= NS - nplain ? 1.0 : a == sq ? sc * sc : sc);
        }
        csum[w][c][ln] = row_sum16(chunk);
    }
    __syncthreads();
    if (t < NS) {
        const int c = t / 16, j = t % 16;
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < NWAVE; ++ww)
#pragma unroll
            for (int r = 0; r < WAVE / 16; ++r) s += csum[ww][c][16 * r + j];
        out[t] = s;
    }
    __syncthreads();
    return M;
}

// Combine per-tile log-domain partials, stored by column: part[c * cs + t]
// for tile t, where column 0 holds the tile max and column 1 + a the tile's
// sum a (a < nsum), scaled by exp(-tile max).  The filter's sums are
// out[a] = sum_t exp(max_t - M) part[1 + a][t] with M = max_t max_t; the
// sum with index sq (a sum of squared weights) scales with exp(2 (max_t - M))
// and the last nplain sums are plain counts, added unscaled.  Every reader
// visits the tiles in a fixed assignment to lanes and a fixed order, so the
// result depends only on ntiles.
//
// General form (any ntiles; many columns): the tile maxima first, then for
// sixteen columns at a time each lane accumulates its tiles' scaled values
// (consecutive lanes read consecutive tiles, so every load is coalesced) and
// the sixteen lane sums are added over the block.
template <int NS>
__device__ __noinline__ double combine_cols(const double* part, int cs, int ntiles, int sq, int nplain, double* out,
                                            double* sh)
{
    constexpr int NCH = (NS + 15) / 16;
    __shared__ double csum[NWAVE][NCH][WAVE];
    double mx = -INFINITY;
    for (int t = threadIdx.x; t < ntiles; t += TILE) mx = fmax(mx, part[t]);
    const double M = block_max(mx, sh);
    const int w = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        double acc[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = 0.0;
        for (int t = threadIdx.x; t < ntiles; t += TILE) {
            const double mt = part[t];
            const double sc = (mt > -INFINITY && M > -INFINITY) ? exp(mt - M) : 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int a = 16 * c + k;
                if (a < NS)
                    acc[k] += (a >= NS - nplain ? 1.0 : a == sq ? sc * sc : sc) * part[(size_t)(1 + a) * cs + t];
            }
        }
        csum[w][c][ln] = row_sum16(acc);
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NS) {
        const int c = t / 16, j = t % 16;
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < NWAVE; ++ww)
#pragma unroll
            for (int r = 0; r < WAVE / 16; ++r) s += csum[ww][c][16 * r + j];
        out[t] = s;
    }
    __syncthreads();
    return M;
}

// The combination for at most 2 TILE tiles and a few columns (the
// first-stage partials; the kinetic and advection-diffusion moments): lane l
// loads tiles l and l + TILE, all their columns at once; the block max of
// the tile maxima; two exponentials per lane; each lane adds its two scaled
// rows; the columns are summed over the block (sixteen at a time with
// row_sum16, or with wave_sum for one column) and across wavefronts in LDS.
// Fixed lane assignment and order, so the result depends only on ntiles.
template <int NS>
__device__ __forceinline__ double combine_pair(const double* part, int cs, int ntiles, int sq, int nplain,
                                               double* out, double* sh)
{
    constexpr int NA = NS + 1;
    constexpr int NCH = (NS + 15) / 16;
    __shared__ double csum[NWAVE][NS == 1 ? 1 : NCH][NS == 1 ? 1 : WAVE];
    const int t0 = threadIdx.x, t1 = t0 + TILE;
    double r0[NA], r1[NA];
    if (t0 < ntiles) {
#pragma unroll
        for (int k = 0; k < NA; ++k) r0[k] = part[(size_t)k * cs + t0];
    } else {
        r0[0] = -INFINITY;
#pragma unroll
        for (int k = 1; k < NA; ++k) r0[k] = 0.0;
    }
    if (t1 < ntiles) {
#pragma unroll
        for (int k = 0; k < NA; ++k) r1[k] = part[(size_t)k * cs + t1];
    } else {
        r1[0] = -INFINITY;
#pragma unroll
        for (int k = 1; k < NA; ++k) r1[k] = 0.0;
    }
    const double M = block_max(fmax(r0[0], r1[0]), sh);
    const double s0 = (r0[0] > -INFINITY && M > -INFINITY) ? exp(r0[0] - M) : 0.0;
    const double s1 = (r1[0] > -INFINITY && M > -INFINITY) ? exp(r1[0] - M) : 0.0;
    auto scale = [&](int a, double r) { return a >= NS - nplain ? 1.0 : a == sq ? r * r : r; };
    const int w = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
    if constexpr (NS == 1) {
        const double v = wave_sum(scale(0, s0) * r0[1] + scale(0, s1) * r1[1]);
        if (ln == 0) csum[w][0][0] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
#pragma unroll
            for (int ww = 0; ww < NWAVE; ++ww) t += csum[ww][0][0];
            out[0] = t;
        }
    } else {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            double chunk[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int a = 16 * c + k;
                chunk[k] = a < NS ? scale(a, s0) * r0[1 + a] + scale(a, s1) * r1[1 + a] : 0.0;
            }
            csum[w][c][ln] = row_sum16(chunk);
        }
        __syncthreads();
        const int t = threadIdx.x;
        if (t < NS) {
            const int c = t / 16, j = t % 16;
            double acc = 0.0;
#pragma unroll
            for (int ww = 0; ww < NWAVE; ++ww)
#pragma unroll
                for (int r = 0; r < WAVE / 16; ++r) acc += csum[ww][c][16 * r + j];
            out[t] = acc;
        }
    }
    __syncthreads();
    return M;
}

// ---------------------------------------------------------------------------
// moments of the parameters for one tile: partial[0] = max l, then
// s0 = sum e, s00 = sum e^2, S1 = sum e d, S2 = sum e d d^T (upper triangle,
// row by row), Sx = sum e x, with e = exp(l - max) and d = theta - c; then
// the NPLAIN counters: the lanes' packed counts, plus the predictor's
// (iterations, fails) of the tile when pred is given (pred[0], pred[cs]),
// and the number of lanes with `neg` set.
// Column c of the tile's partials goes to out_part[c * cs].  P and D are the
// model's, so every register index is static.
// ---------------------------------------------------------------------------
template <class R, int P, int D>
__device__ void tile_moments(double l, bool valid, const double* th, const R* x, const double* cshift,
                             uint64_t counts, const double* pred, double* out_part, int cs, double* sh,
                             bool neg = false)
{
    constexpr int NV = 2 + P + P * (P + 1) / 2 + D;   // weighted sums
    constexpr int NCH = (NV + 15) / 16;
    __shared__ double part[NWAVE][NCH][WAVE];
    __shared__ double cw[NWAVE][4];
    const double lv = valid ? l : -INFINITY;
    const double Mt = block_max(lv, sh);
    const double e = (valid && lv > -INFINITY) ? exp(lv - Mt) : 0.0;
    double dv[P];
#pragma unroll
    for (int i = 0; i < P; ++i) dv[i] = e > 0.0 ? th[i] - cshift[i] : 0.0;
    double v[NCH * 16];
    v[0] = e;
    v[1] = e * e;
#pragma unroll
    for (int i = 0; i < P; ++i) v[2 + i] = e * dv[i];
#pragma unroll
    for (int i = 0, k = 2 + P; i < P; ++i)
#pragma unroll
        for (int j = i; j < P; ++j, ++k) v[k] = e * dv[i] * dv[j];
#pragma unroll
    for (int i = 0; i < D; ++i) v[2 + P + P * (P + 1) / 2 + i] = e > 0.0 ? e * (double)x[i] : 0.0;
#pragma unroll
    for (int k = NV; k < NCH * 16; ++k) v[k] = 0.0;
    const int w = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        double chunk[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) chunk[k] = v[16 * c + k];
        part[w][c][ln] = row_sum16(chunk);
    }
    const uint64_t wc = wave_sum_u64(counts);
    const uint64_t wneg = __ballot(neg);
    if (ln == 0) {
        cw[w][0] = count_iters(wc);
        cw[w][1] = count_fails(wc);
        cw[w][2] = count_nonf(wc);
        cw[w][3] = (double)__popcll(wneg);
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NV + NPLAIN) {
        double s = 0.0;
        if (t < NV) {
            const int c = t / 16, j = t % 16;
#pragma unroll
            for (int ww = 0; ww < NWAVE; ++ww)
#pragma unroll
                for (int r = 0; r < WAVE / 16; ++r) s += part[ww][c][16 * r + j];
        } else {
            const int k = t - NV;
            if (k < 3 || k == 4) {
                const int kc = k < 3 ? k : 3;
#pragma unroll
                for (int ww = 0; ww < NWAVE; ++ww) s += cw[ww][kc];
            }
            if (pred && k == 1) s += pred[cs];
            if (pred && k == 3) s += pred[0];
        }
        out_part[(size_t)(1 + t) * cs] = s;
    }
    if (threadIdx.x == 0) out_part[0] = Mt;
    __syncthreads();
}

// Last step of a moment pass, in one lane with the model's P and D known at
// compile time (so every array lives in registers): mean, covariance,
// ESS, state mean, and the Cholesky factor with the jitter rule (retry with
// C + delta I, delta = 1e-10 tr(C)/p, then 10x larger, at most five times).
// The factor overwrites a packed lower triangle of C (row i at i(i+1)/2).
// Commits unless degenerate; `flip` switches to the new ensemble buffers and
// advances the step counter.
// State fields a moment pass reads, loaded before the tile combine so that
// the loads overlap it (the moments kernel is one workgroup per filter and
// latency bound).
struct MomPre {
    double tb[PMAX];
    double t;
    uint64_t j, T;
    unsigned long long jit, n_pred, n_upd, n_fail, n_nonf, n_neg;
    int32_t cur;
};
template <int P>
__device__ inline MomPre mom_prefetch(const FilterState& st)
{
    MomPre r;
#pragma unroll
    for (int i = 0; i < P; ++i) r.tb[i] = st.theta_bar[i];
    r.t = st.t;
    r.j = st.j;
    r.T = st.T;
    r.jit = st.jitters;
    r.n_pred = st.newton_pred;
    r.n_upd = st.newton_upd;
    r.n_fail = st.newton_fails;
    r.n_nonf = st.nonfinite;
    r.n_neg = st.negative;
    r.cur = st.cur;
    return r;
}

template <int P, int D>
__device__ __forceinline__ int32_t moments_tail(const double* tot, const MomPre& pre, FilterState& st, bool flip,
                                                double t_next)
{
    constexpr int NT = P * (P + 1) / 2;
    const double s0 = tot[0], s00 = tot[1];
    if (!(s0 > 0.0) || !isfinite(s0)) return ST_EDEGENERATE;
    const double inv = 1.0 / s0;
    double dm[P];
#pragma unroll
    for (int i = 0; i < P; ++i) dm[i] = tot[2 + i] * inv;
    // tot holds the upper triangle row by row: entry (i, j), j >= i, sits at
    // 2 + P + i*P - i*(i-1)/2 + (j - i)
    auto cov = [&](int i, int j) -> double {
        const int r = i < j ? i : j, c = i < j ? j : i;
        return tot[2 + P + r * P - r * (r - 1) / 2 + (c - r)] * inv - dm[i] * dm[j];
    };
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) tr += cov(i, i);
    double L[NT];
    double delta = 0.0;
    int jit = -1;
    for (int attempt = 0; attempt <= 5 && jit < 0; ++attempt) {
        if (attempt == 1) delta = 1e-10 * tr / P;
        else if (attempt > 1) delta *= 10.0;
        bool ok = true;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            double sdiag = cov(j, j) + delta;
#pragma unroll
            for (int k = 0; k < j; ++k) sdiag -= L[j * (j + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
            ok = ok && sdiag > 0.0 && isfinite(sdiag);
            const double ljj = sqrt(ok ? sdiag : 1.0);
            const double rl = 1.0 / ljj;
            L[j * (j + 1) / 2 + j] = ljj;
#pragma unroll
            for (int i = j + 1; i < P; ++i) {
                double t = cov(i, j);
#pragma unroll
                for (int k = 0; k < j; ++k) t -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
                L[i * (i + 1) / 2 + j] = t * rl;
            }
        }
        if (ok) jit = attempt;
    }
    if (jit < 0) return ST_EDEGENERATE;
#pragma unroll
    for (int i = 0; i < P; ++i) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            st.C[i * P + j] = cov(i, j);
            st.L[i * P + j] = j <= i ? L[i * (i + 1) / 2 + j] : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < P; ++i) st.theta_bar[i] = pre.tb[i] + dm[i];
#pragma unroll
    for (int i = 0; i < D; ++i) st.state_mean[i] = tot[2 + P + NT + i] * inv;
    st.ess = s0 * s0 / s00;
    st.jitters = pre.jit + (unsigned long long)jit;
    if (flip) {
        st.cur = pre.cur ^ 1;
        st.j = pre.j + 1;
        st.t = t_next;
    }
    return ST_OK;
}


// Moment pass of one filter (one workgroup): the tile combine, then in lane
// 0 the counters and the tail.  The combine only reads, so callers run it
// before deciding whether the step commits.
template <int P, int D>
__device__ __forceinline__ void moments_combine(const FilterDesc& fd, double* tot, double* sh)
{
    constexpr int NA = 1 + 2 + P + P * (P + 1) / 2 + D + NPLAIN;
    if constexpr (NA * 8 <= 256) {
        if (fd.ntiles <= 2 * TILE) combine_pair<NA - 1>(fd.part2, fd.ntiles, fd.ntiles, 1, NPLAIN, tot, sh);
        else combine_rows<NA - 1>(fd.part2, fd.ntiles, fd.ntiles, 1, NPLAIN, tot, sh);
    } else {
        if (fd.ntiles <= TILE) combine_wide<NA - 1>(fd.part2, fd.ntiles, fd.ntiles, 1, NPLAIN, tot, sh);
        else combine_cols<NA - 1>(fd.part2, fd.ntiles, fd.ntiles, 1, NPLAIN, tot, sh);
    }
}
// The same tail for larger P with the whole workgroup: covariance entries in
// parallel, then a right-looking Cholesky in LDS, one column per round (the
// column scaled by 1/l_jj, then the trailing triangle updated in parallel).
// Every entry sees the same operations in the same order as in moments_tail
// (c_ij + delta - l_i0 l_j0 - l_i1 l_j1 - ..., then times 1/l_jj), and so
// does the jitter rule; a failed column ends an attempt early.
template <int P, int D>
__device__ __forceinline__ int32_t moments_tail_wg(const double* tot, const MomPre& pre, FilterState& st, bool flip,
                                                   double t_next)
{
    constexpr int NT = P * (P + 1) / 2;
    __shared__ double cv[P][P];
    __shared__ double A[P][P];
    __shared__ double dms[P];
    const int t = threadIdx.x;
    const double s0 = tot[0], s00 = tot[1];
    if (!(s0 > 0.0) || !isfinite(s0)) return ST_EDEGENERATE;
    const double inv = 1.0 / s0;
    if (t < P) dms[t] = tot[2 + t] * inv;
    __syncthreads();
    for (int e = t; e < P * P; e += TILE) {
        const int i = e / P, j = e % P;
        const int r = i < j ? i : j, c = i < j ? j : i;
        cv[i][j] = tot[2 + P + r * P - r * (r - 1) / 2 + (c - r)] * inv - dms[i] * dms[j];
    }
    __syncthreads();
    // the factorisation runs in wavefront 0 alone: its rounds order their LDS
    // traffic with wavefront-scope fences instead of workgroup barriers
    __shared__ int jit_sh;
    if (t < WAVE) {
        double tr = 0.0;
#pragma unroll
        for (int i = 0; i < P; ++i) tr += cv[i][i];
        double delta = 0.0;
        int jit = -1;
        for (int attempt = 0; attempt <= 5 && jit < 0; ++attempt) {
            if (attempt == 1) delta = 1e-10 * tr / P;
            else if (attempt > 1) delta *= 10.0;
            for (int e = t; e < P * P; e += WAVE) {
                const int i = e / P, j = e % P;
                A[i][j] = i == j ? cv[i][j] + delta : cv[i][j];
            }
            wave_sync();
            bool ok = true;
            for (int j = 0; j < P && ok; ++j) {
                const double sdiag = A[j][j];
                ok = sdiag > 0.0 && isfinite(sdiag);
                if (ok) {
                    const double ljj = sqrt(sdiag);
                    const double rl = 1.0 / ljj;
                    wave_sync();
                    if (t == j) A[j][j] = ljj;
                    if (t > j && t < P) A[t][j] = A[t][j] * rl;
                    wave_sync();
                    // trailing triangle: rows i > j, columns j < k <= i
                    const int m = P - j - 1;
                    for (int e = t; e < m * (m + 1) / 2; e += WAVE) {
                        int i = 0;
                        while ((i + 1) * (i + 2) / 2 <= e) ++i;
                        const int k = e - i * (i + 1) / 2;
                        const int ii = j + 1 + i, kk = j + 1 + k;
                        A[ii][kk] -= A[ii][j] * A[kk][j];
                    }
                    wave_sync();
                }
            }
            if (ok) jit = attempt;
        }
        if (t == 0) jit_sh = jit;
    }
    __syncthreads();
    const int jit = jit_sh;
    if (jit < 0) return ST_EDEGENERATE;
    for (int e = t; e < P * P; e += TILE) {
        const int i = e / P, j = e % P;
        st.C[e] = cv[i][j];
        st.L[e] = j <= i ? A[i][j] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < P; ++i)   // static indices keep pre in registers
        if (t == i) st.theta_bar[i] = pre.tb[i] + dms[i];
    if (t < D) st.state_mean[t] = tot[2 + P + NT + t] * inv;
    if (t == 0) {
        st.ess = s0 * s0 / s00;
        st.jitters = pre.jit + (unsigned long long)jit;
        if (flip) {
            st.cur = pre.cur ^ 1;
            st.j = pre.j + 1;
            st.t = t_next;
        }
    }
    return ST_OK;
}

// counters of the step from the counter columns of the combined partials
__device__ __forceinline__ void moments_counters(const FilterDesc& fd, const double* tot, const MomPre& pre,
                                                 FilterState& st)
{
    const double* c = tot + fd.nacc - 1 - NPLAIN;
    st.newton_upd = pre.n_upd + (unsigned long long)c[0];
    st.newton_fails = pre.n_fail + (unsigned long long)c[1];
    st.nonfinite = pre.n_nonf + (unsigned long long)c[2];
    st.newton_pred = pre.n_pred + (unsigned long long)c[3];
    st.negative = pre.n_neg + (unsigned long long)c[4];
}

// counters and tail, called by the whole workgroup; returns the status to
// every thread.  Small P: one lane; larger P: the workgroup.
template <int P, int D>
__device__ __forceinline__ int32_t moments_finish(const FilterDesc& fd, const double* tot, const MomPre& pre,
                                                  FilterState& st, bool flip, double t_next)
{
    __shared__ int32_t status;
    if (threadIdx.x == 0) moments_counters(fd, tot, pre, st);
    if constexpr (P >= 8) {
        return moments_tail_wg<P, D>(tot, pre, st, flip, t_next);
    } else {
        if (threadIdx.x == 0) status = moments_tail<P, D>(tot, pre, st, flip, t_next);
        __syncthreads();
        return status;
    }
}

// ---------------------------------------------------------------------------
// common item decode and step validity
// ---------------------------------------------------------------------------
struct Item {
    int b, slot, tile;
    StepRec rec;
};
// items, batch entries and slots are uniform over the workgroup; saying so
// lets the compiler use scalar loads for every descriptor field
__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// INL: the inline (single-filter) form of the batch, a compile-time choice
// so that every record and descriptor read is a scalar load
template <bool INL>
__device__ inline StepRec record(const Batch& B, int b)
{
    if constexpr (INL) return B.one;
    else return B.recs[b];
}

// The tile of workgroup w when a single filter's kernel runs one workgroup
// per tile: workgroups go to the eight XCDs in turn (XCD w mod 8), so XCD x
// takes the contiguous tiles [x q + min(x, r), ...) with nt = 8 q + r, as
// many as it has workgroups.  A tile's neighbours (its slots' ancestors and
// the prefix tiles their search reads) then sit in the same XCD's L2, in
// every kernel of the step.  A bijection on [0, nt); results do not depend
// on which workgroup runs a tile.
__device__ inline int xcd_tile(int w, int nt)
{
    const int x = w % 8, q = nt / 8, r = nt % 8;
    return x * q + (x < r ? x : r) + w / 8;
}

template <bool INL>
__device__ inline Item fetch(const Batch& B, int itx)
{
    Item r;
    if constexpr (INL) {
        r.b = 0;
        r.tile = (int)gridDim.x == B.fd.ntiles ? xcd_tile(itx, B.fd.ntiles) : itx;
        r.rec = B.one;
    } else {
        const uint32_t it = (uint32_t)uniform((int)B.items[itx]);
        r.b = (int)(it >> 16);
        r.tile = (int)(it & 0xFFFFu);
        r.rec = B.recs[r.b];
    }
    r.slot = uniform(r.rec.slot);
    return r;
}

template <bool INL>
__device__ inline const FilterDesc& desc_of(const Batch& B, const FilterDesc* descs, int slot)
{
    if constexpr (INL) return B.fd;
    else return descs[slot];
}

// The step of batch entry b may run: its observation time is after the
// filter's current time (checked again, identically, by every kernel; the
// final kernel reports PF_EORDER).
__device__ inline bool step_valid(const StepRec& r, const FilterState& st) { return r.t_next > st.t; }

// Uniform values loaded together with the ones a branch tests: an empty asm
// that takes them in scalar registers keeps the compiler from sinking their
// loads below the branch (a second round trip to memory before the first use).
template <class T>
__device__ __forceinline__ void keep_loaded(const T v)
{
    asm volatile("" ::"s"(v));
}
template <class T, class... U>
__device__ __forceinline__ void keep_loaded(const T v, const U... rest)
{
    keep_loaded(v);
    keep_loaded(rest...);
}

// ---------------------------------------------------------------------------
// the step-4 normals of one output slot (Algorithm 1 steps 4(a) and 4(d)):
// they depend only on (seed, step, slot), so they are drawn ahead of the
// update kernel, where workgroups are idle, into the filter's z buffer; the
// update kernel takes them from there when the tile's tag names its step and
// draws them itself otherwise
// ---------------------------------------------------------------------------
template <class R, int P, int D>
__device__ inline void draw_slot_normals(const FilterDesc& fd, uint64_t step, int n)
{
    R z[P], zi[D];
    normals<P, R>(fd.seed, step, (uint64_t)n, PUR_PROLIF, z);
    normals<D, R>(fd.seed, step, (uint64_t)n, PUR_INNOV, zi);
    R* zb = (R*)fd.z;
#pragma unroll
    for (int i = 0; i < P; ++i) zb[(size_t)i * fd.npad + n] = z[i];
#pragma unroll
    for (int i = 0; i < D; ++i) zb[(size_t)(P + i) * fd.npad + n] = zi[i];
}

// the slots of tile pairs (2 (blockIdx.x - first), + 1), stepping by
// gridDim.x - first pairs, for `step`: each lane draws for one slot in each
// tile of the pair, two independent generators the compiler interleaves
// (half the wavefronts of one per slot, at the same arithmetic).  A tile's
// tag follows its normals; both are read by a later kernel, after this one
// has completed.
template <class R, int P, int D>
__device__ inline void draw_pair(const FilterDesc& fd, uint64_t step, int n0, int n1)
{
    R z0[P], z1[P], i0[D], i1[D];
    normals<P, R>(fd.seed, step, (uint64_t)n0, PUR_PROLIF, z0);
    normals<P, R>(fd.seed, step, (uint64_t)n1, PUR_PROLIF, z1);
    normals<D, R>(fd.seed, step, (uint64_t)n0, PUR_INNOV, i0);
    normals<D, R>(fd.seed, step, (uint64_t)n1, PUR_INNOV, i1);
    R* zb = (R*)fd.z;
    if (n0 < fd.n) {
#pragma unroll
        for (int i = 0; i < P; ++i) zb[(size_t)i * fd.npad + n0] = z0[i];
#pragma unroll
        for (int i = 0; i < D; ++i) zb[(size_t)(P + i) * fd.npad + n0] = i0[i];
    }
    if (n1 < fd.n) {
#pragma unroll
        for (int i = 0; i < P; ++i) zb[(size_t)i * fd.npad + n1] = z1[i];
#pragma unroll
        for (int i = 0; i < D; ++i) zb[(size_t)(P + i) * fd.npad + n1] = i1[i];
    }
}

template <class Model>
__device__ inline void draw_ahead(const FilterDesc& fd, uint64_t step, int first)
{
    constexpr int P = Model::P, D = Model::D;
    for (int t0 = 2 * (blockIdx.x - first); t0 < fd.ntiles; t0 += 2 * (gridDim.x - first)) {
        const int n0 = t0 * TILE + threadIdx.x, n1 = n0 + TILE;
        if (fd.prec == PREC_FP32) draw_pair<float, P, D>(fd, step, n0, n1);
        else draw_pair<double, P, D>(fd, step, n0, n1);
        if (threadIdx.x == 0) {
            fd.ztag[t0] = step;
            if (t0 + 1 < fd.ntiles) fd.ztag[t0 + 1] = step;
        }
    }
}

// ---------------------------------------------------------------------------
// step 1: prior draw and initial moment partials
// ---------------------------------------------------------------------------
template <class Model, class R>
__global__ __launch_bounds__(TILE) void k_init(int slot, const FilterDesc* descs, FilterState* states)
{
    constexpr int D = Model::D, P = Model::P;
    __shared__ double sh[TILE];
    const FilterDesc& fd = descs[slot];
    for (int tile = blockIdx.x; tile < fd.ntiles; tile += gridDim.x) {
        const int n = tile * TILE + threadIdx.x;
        const bool valid = n < fd.n;
        double th[P];
        R xs[D];
#pragma unroll
        for (int i = 0; i < P; ++i) th[i] = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) xs[i] = R(0);
        if (valid) {
            double z[P];
            normals<P>(fd.seed, 0, (uint64_t)n, PUR_PRIOR, z);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                th[i] = fd.prior_mean[i] + fd.prior_sd[i] * z[i];
                fd.theta[0][(size_t)i * fd.npad + n] = th[i];
            }
            R* x = (R*)fd.x[0];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                xs[i] = (R)fd.x0[i];
                x[(size_t)i * fd.npad + n] = xs[i];
            }
            fd.logw[0][n] = -log((double)fd.n);
        }
        tile_moments<R, P, D>(-log((double)fd.n), valid, th, xs, fd.prior_mean, 0, nullptr, fd.part2 + tile,
                              fd.ntiles, sh);
        // the first observation step's normals
        if (fd.z) {
            if (valid) draw_slot_normals<R, P, D>(fd, 1, n);
            if (threadIdx.x == 0) fd.ztag[tile] = 1;
        }
    }
}

// one workgroup: moments of the prior draw (the shift is the prior mean, which
// the host stored as theta_bar)
template <class Model>
__global__ __launch_bounds__(TILE) void k_init_moments(int slot, const FilterDesc* descs, FilterState* states)
{
    constexpr int P = Model::P, D = Model::D;
    __shared__ double sh[TILE];
    __shared__ double tot[NACC_MAX];
    const FilterDesc& fd = descs[slot];
    FilterState& st = states[slot];
    const MomPre pre = mom_prefetch<P>(st);
    moments_combine<P, D>(fd, tot, sh);
    const int32_t status = moments_finish<P, D>(fd, tot, pre, st, false, pre.t);
    if (threadIdx.x == 0) st.status = status;
}

// ---------------------------------------------------------------------------
// steps 2 and 3(a): shrink, predictor, first-stage log-weights
// ---------------------------------------------------------------------------
template <class Model, class R, int KORD, int LMM, bool INL>
__global__ __launch_bounds__(TILE) void k_predict(Batch B, const FilterDesc* __restrict__ descs, FilterState* __restrict__ states)
{
    constexpr int D = Model::D, P = Model::P;
    __shared__ double sh[TILE];
    __shared__ unsigned long long wcnt[NWAVE];
    for (int itx = blockIdx.x; itx < B.n_items; itx += gridDim.x) {
        const Item itm = fetch<INL>(B, itx);
        const StepRec& rec = itm.rec;
        const FilterDesc& fd = desc_of<INL>(B, descs, itm.slot);
        const FilterState& st = states[itm.slot];
        // the state fields and buffer pointers, loaded before the test waits
        const double t_cur = st.t;
        const int cur = st.cur;
        const R* const xb = (const R*)(cur ? fd.x[1] : fd.x[0]);
        const double* const tb = cur ? fd.theta[1] : fd.theta[0];
        const double* const lw = cur ? fd.logw[1] : fd.logw[0];
        keep_loaded(xb, tb, lw);
        if (!(rec.t_next > t_cur)) continue;
        const double h = (rec.t_next - t_cur) / fd.substeps;
        const int n = itm.tile * TILE + threadIdx.x;
        const bool valid = n < fd.n;
        double lg = -INFINITY;
        uint32_t iters = 0, fails = 0;
        if (valid) {
            R x[D];
#pragma unroll
            for (int i = 0; i < D; ++i) x[i] = xb[(size_t)i * fd.npad + n];
            double m[P];
            const double a = fd.a;
#pragma unroll
            for (int i = 0; i < P; ++i)
                m[i] = a * tb[(size_t)i * fd.npad + n] + (1.0 - a) * st.theta_bar[i];
            Model md;
            md.set_params(m, fd);
            const R* fl = sizeof(R) == 4 ? (const R*)fd.floor_f : (const R*)fd.floor_;
            integrate_lmm<Model, R, KORD, false, LMM>(md, x, nullptr, h, fd.substeps, (R)fd.rtol, fl, fd.kmax,
                                             iters, fails);
            const double lb = loglik<R>(x, fd.obs, rec.y, rec.sigma, fd.m);
            lg = lw[n] + lb;
            if (!(lg > -INFINITY)) lg = -INFINITY;   // NaN -> zero weight
            fd.lbar[n] = lb;
            fd.lg[n] = lg;
        }
        // per-wavefront counts: written before the barriers of block_max,
        // read before those of block_sum (which the next tile's writes follow)
        const uint64_t wc = wave_sum_u64(pack_counts(iters, fails, 0));
        if (threadIdx.x % WAVE == 0) wcnt[threadIdx.x / WAVE] = wc;
        const double Mt = block_max(lg, sh);
        double ci = 0.0, cf = 0.0;
        if (threadIdx.x == 0) {
#pragma unroll
            for (int w = 0; w < NWAVE; ++w) {
                ci += count_iters(wcnt[w]);
                cf += count_fails(wcnt[w]);
            }
        }
        const double e = lg > -INFINITY ? exp(lg - Mt) : 0.0;
        const double s = block_sum(e, sh);
        if (threadIdx.x == 0) {
            double* p1 = fd.part1 + itm.tile;
            const size_t cs = (size_t)fd.ntiles;
            p1[0] = Mt;
            p1[cs] = s;
            p1[2 * cs] = ci;
            p1[3 * cs] = cf;
        }
    }
}

// ---------------------------------------------------------------------------
// step 3(b): systematic resampling in integers
// ---------------------------------------------------------------------------
template <bool INL>
__global__ __launch_bounds__(TILE) void k_count(Batch B, const FilterDesc* __restrict__ descs, FilterState* __restrict__ states)
{
    __shared__ double sh[TILE];
    __shared__ double tot[1];
    __shared__ unsigned long long shu[NWAVE];
    for (int itx = blockIdx.x; itx < B.n_items; itx += gridDim.x) {
        const Item itm = fetch<INL>(B, itx);
        const FilterDesc& fd = desc_of<INL>(B, descs, itm.slot);
        FilterState& st = states[itm.slot];
        // every load is issued before anything waits: the lane's log-weight,
        // the filter state (the step's validity only gates the stores), and
        // the tile partials of the combine
        const int n = itm.tile * TILE + threadIdx.x;
        const double l = n < fd.n ? fd.lg[n] : -INFINITY;
        const double t_cur = st.t;
        const uint64_t j_cur = st.j, v_test = st.V;
        double M = 0.0, S = 1.0;
        if (!fd.g_direct) {
            // the filter's first-stage log-sum-exp, from the tile partials
            M = fd.ntiles <= 2 * TILE ? combine_pair<1>(fd.part1, fd.ntiles, fd.ntiles, -1, 0, tot, sh)
                                      : combine_rows<1>(fd.part1, fd.ntiles, fd.ntiles, -1, 0, tot, sh);
            S = tot[0];
        }
        const bool ok = fd.g_direct || (M > -INFINITY && isfinite(M) && S > 0.0);
        unsigned long long q = 0;
        if (n < fd.n) {
            const double g = fd.g_direct ? l : (ok && l > -INFINITY ? exp(l - M) / S : 0.0);
            if (g > 0.0) q = (unsigned long long)floor(ldexp(g, fd.shift));
        }
        // the inclusive prefix of q within the tile (every lane of the tile,
        // so the prefix is monotone up to lane 255) and the tile's sum
        unsigned long long ex;
        const unsigned long long ts = block_exscan_u64(q, ex, shu);
        if (!fd.g_direct && !(itm.rec.t_next > t_cur)) continue;   // the step does not run
        fd.q[n] = ex + q;
        if (threadIdx.x == 0) fd.tsum[itm.tile] = ts;
        if (itm.tile == 0 && threadIdx.x == 0) {
            // the systematic draw's one uniform word of the filter and step,
            // drawn once here for the scatter (test mode: the host's)
            if (fd.resampling == 0) {
                uint64_t r = v_test;
                if (!fd.g_direct) {
                    uint64_t w[4];
                    Philox::block(j_cur + 1, 0, PUR_RESAMPLE, 0, fd.seed, 0, w);
                    r = w[0];
                }
                st.R = r;
            }
            st.j_run = j_cur + 1;
        }
    }
}

// first output slot of the copies of a particle whose inclusive cumulative
// integer weight is c: F(c) = min(N, ceil((c N - V) / T)) if c N > V, else 0
__device__ inline uint64_t first_slot(uint64_t c, uint64_t N, uint64_t T, uint64_t V)
{
    const uint64_t cn = c * N;
    if (cn <= V) return 0;
    const uint64_t f = (cn - V + T - 1) / T;
    return f < N ? f : N;
}

// copies of one particle written by its own lane up to this many; longer
// runs (a few heavy particles when the weights are very uneven) are written
// by the whole workgroup
constexpr uint64_t LONG_RUN = 16;

// Multinomial draw for the output slots of one tile (Algorithm 1 step 3(b)
// literally): the filter's tile offsets P (exclusive prefix of the tile sums,
// P[ntiles] = T) are built in LDS by every workgroup in the same order; slot
// i draws tau_i = floor(r_i T / 2^64) from its own RESAMPLE word, finds the
// tile s with P[s] <= tau_i < P[s+1] by bisection in LDS, then the particle by
// bisection over that tile's inclusive prefix (written by k_count).
// The filter's tile offsets in LDS: P[s] = the exclusive prefix of the tile
// sums, P[ntiles] = T, built by every workgroup in the same order (exact
// integers, so any order gives the same values).  MAXT tile sums at most.
template <int MAXT>
__device__ inline unsigned long long tile_offsets(const FilterDesc& fd, unsigned long long* P,
                                                  unsigned long long* shu)
{
    const int nt = fd.ntiles;
    constexpr int PER = MAXT / TILE;   // tile sums per lane
    unsigned long long v[PER], loc = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x * PER + k;
        v[k] = t < nt ? fd.tsum[t] : 0ull;
        loc += v[k];
    }
    unsigned long long ex;
    const unsigned long long T = block_exscan_u64(loc, ex, shu);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x * PER + k;
        if (t < nt) P[t] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) P[nt] = T;
    __syncthreads();
    return T;
}

__device__ inline void multinomial_tile(const FilterDesc& fd, FilterState& st, int tile, uint64_t step, bool run,
                                        unsigned long long* P, unsigned long long* shu)
{
    const int nt = fd.ntiles;
    const unsigned long long T = tile_offsets<MULTI_MAX_TILES>(fd, P, shu);
    if (!run) return;
    if (tile == 0 && threadIdx.x == 0) {
        st.T = T;
        st.V = 0;
    }
    const int i = tile * TILE + threadIdx.x;
    if (T == 0 || i >= fd.n) return;
    uint64_t w[4];
    Philox::block(step, (uint64_t)i, PUR_RESAMPLE, 0, fd.seed, 0, w);
    const uint64_t tau = __umul64hi(w[0], T);
    int lo = 0, hi = nt;   // last s with P[s] <= tau  (P[0] = 0 <= tau < P[nt] = T)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (P[mid] <= tau) lo = mid;
        else hi = mid;
    }
    const uint64_t rem = tau - P[lo];
    const uint64_t* cq = fd.q + (size_t)lo * TILE;
    int a = 0, b = TILE - 1;   // first k with cq[k] > rem (cq[255] = tile sum > rem)
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (cq[mid] > rem) b = mid;
        else a = mid + 1;
    }
    fd.anc[i] = lo * TILE + a;
}

template <bool INL>
__global__ __launch_bounds__(TILE) void k_scatter(Batch B, const FilterDesc* descs, FilterState* states)
{
    __shared__ unsigned long long P[MULTI_MAX_TILES + 1];
    __shared__ unsigned long long shu[2 * NWAVE];
    __shared__ int n_long;
    __shared__ uint32_t run_lo[TILE], run_hi[TILE];
    __shared__ int run_k[TILE];
    for (int itx = blockIdx.x; itx < B.n_items; itx += gridDim.x) {
        const Item itm = fetch<INL>(B, itx);
        const FilterDesc& fd = desc_of<INL>(B, descs, itm.slot);
        FilterState& st = states[itm.slot];
        if (fd.resampling == 1) {
            const bool run = fd.g_direct || itm.rec.t_next > st.t;
            multinomial_tile(fd, st, itm.tile, st.j + 1, run, P, shu);
            __syncthreads();
            continue;
        }
        // loads first: this lane's weight and exclusive offset within the
        // tile (from the count pass's inclusive prefix), the filter state, the
        // tile sums (the step's validity only gates the stores)
        const int n = itm.tile * TILE + threadIdx.x;
        const unsigned long long ex = threadIdx.x > 0 ? fd.q[n - 1] : 0ull;
        const unsigned long long q = n < fd.n ? fd.q[n] - ex : 0ull;
        // exclusive offset of this tile and total T of the integer weights:
        // the first two tile sums of each lane are loaded with the rest, so
        // one round trip covers up to 2 TILE tiles (2 TILE^2 particles)
        const int nt = fd.ntiles;
        const int t0 = threadIdx.x, t1 = t0 + TILE;
        const unsigned long long v0 = t0 < nt ? fd.tsum[t0] : 0ull;
        const unsigned long long v1 = t1 < nt ? fd.tsum[t1] : 0ull;
        const double t_cur = st.t;
        const uint64_t r = st.R;   // the step's uniform word, from the count pass
        unsigned long long all = v0 + v1;
        unsigned long long pre = (t0 < itm.tile ? v0 : 0ull) + (t1 < itm.tile ? v1 : 0ull);
        for (int t = t0 + 2 * TILE; t < nt; t += TILE) {
            const unsigned long long v = fd.tsum[t];
            all += v;
            if (t < itm.tile) pre += v;
        }
        unsigned long long T;
        block_sum2_u64(pre, all, shu, pre, T);
        if (!fd.g_direct && !(itm.rec.t_next > t_cur)) continue;   // the step does not run
        const uint64_t V = T ? __umul64hi(r, T) : 0;
        if (itm.tile == 0 && threadIdx.x == 0) {
            st.T = T;
            if (!fd.g_direct) st.V = V;
        }
        if (T == 0) continue;
        if (threadIdx.x == 0) n_long = 0;
        __syncthreads();
        if (q > 0) {
            const uint64_t N = (uint64_t)fd.n;
            const uint64_t lo_c = pre + ex;
            const uint64_t lo = first_slot(lo_c, N, T, V);
            const uint64_t hi = first_slot(lo_c + q, N, T, V);
            if (hi - lo <= LONG_RUN) {
                for (uint64_t i = lo; i < hi; ++i) fd.anc[i] = n;
            } else {
                // a heavy particle: the whole workgroup writes its copies below
                const int e = atomicAdd(&n_long, 1);
                run_lo[e] = (uint32_t)lo;
                run_hi[e] = (uint32_t)hi;
                run_k[e] = n;
            }
        }
        __syncthreads();
        for (int e = 0; e < n_long; ++e)
            for (uint32_t i = run_lo[e] + threadIdx.x; i < run_hi[e]; i += TILE) fd.anc[i] = run_k[e];
    }
}

// A single kinetic filter's systematic draw is folded into its update
// kernel (no scatter pass) when its tile offsets fit in LDS.  Host and device
// decide it the same way.
constexpr int FOLD_MAX_TILES = 2048;   // N <= 2^19
__host__ __device__ inline bool fold_scatter(const FilterDesc& fd)
{
    return fd.model != MODEL_ADVDIFF && fd.resampling == 0 && !fd.g_direct && fd.ntiles <= FOLD_MAX_TILES;
}

// The systematic draw's slot assignment from the slot side: output slot i
// takes the first particle k with C_k N > u_i = i T + V, C the cumulative
// integer weights -- the same assignment as the scatter pass's
// F(C_{k-1}) <= i < F(C_k).  Every product is below 2^63 (i T < N 2^shift
// <= 2^62, C_k N <= T N).  First the tile: the last s with P[s] N <= u
// (bisection over the LDS offsets; P[ntiles] N > u).
__device__ inline int offset_tile(const unsigned long long* P, int ntiles, uint64_t N, uint64_t u)
{
    int lo = 0, hi = ntiles;   // P[lo] N <= u < P[hi] N
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (P[mid] * N <= u) lo = mid;
        else hi = mid;
    }
    return lo;
}

// then the particle within tile s, from the tile's inclusive prefix cq
// (base = P[s]; its last entry ends above u): from LDS by bisection ...
__device__ inline int intile_lds(const unsigned long long* cq, uint64_t base, uint64_t N, uint64_t u)
{
    int a = 0, b = TILE - 1;   // first k with (base + cq[k]) N > u
    while (a < b) {
        const int mid = (a + b) >> 1;
        if ((base + cq[mid]) * N > u) b = mid;
        else a = mid + 1;
    }
    return a;
}

// ... or from global memory in two rounds of sixteen independent loads (the
// ends of the tile's sixteen blocks, then the chosen block's entries)
__device__ inline int intile_global(const uint64_t* cq, uint64_t base, uint64_t N, uint64_t u)
{
    uint64_t ends[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) ends[j] = cq[16 * j + 15];
    int b = 0;   // blocks that end at or below u (the last one ends above)
#pragma unroll
    for (int j = 0; j < 15; ++j) b += (base + ends[j]) * N <= u ? 1 : 0;
    uint64_t c[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) c[j] = cq[16 * b + j];
    int k = 0;
#pragma unroll
    for (int j = 0; j < 15; ++j) k += (base + c[j]) * N <= u ? 1 : 0;
    return 16 * b + k;
}

// tiles of prefixes a workgroup stages in LDS when its slots' ancestors lie
// in that few (else each lane searches global memory)
constexpr int FOLD_STAGE = 4;

// ---------------------------------------------------------------------------
// steps 3(c)-5 per output slot
// ---------------------------------------------------------------------------
template <class Model, class R, int KORD, int LMM, bool INL>
__global__ __launch_bounds__(TILE) void k_update(Batch B, const FilterDesc* __restrict__ descs, FilterState* __restrict__ states)
{
    constexpr int D = Model::D, P = Model::P;
    __shared__ double sh[TILE];
    // the folded systematic draw's tile offsets (single-filter form only)
    __shared__ unsigned long long Poff[INL ? FOLD_MAX_TILES + 1 : 1];
    __shared__ unsigned long long cqs[INL ? FOLD_STAGE * TILE : 1];
    __shared__ unsigned long long shu[NWAVE];
    __shared__ int lo_sh[2];
    for (int itx = blockIdx.x; itx < B.n_items; itx += gridDim.x) {
        const Item itm = fetch<INL>(B, itx);
        const StepRec& rec = itm.rec;
        const FilterDesc& fd = desc_of<INL>(B, descs, itm.slot);
        FilterState& st = states[itm.slot];
        const int n = itm.tile * TILE + threadIdx.x;
        const bool valid = n < fd.n;
        const bool fold = INL && fold_scatter(fd);
        int k_anc = valid && !fold ? fd.anc[n] : 0;   // issued before the state checks wait
        const uint64_t ztag = fd.ztag ? fd.ztag[itm.tile] : 0;
        // every state field the step reads, loaded before any test waits on one
        const double t_cur = st.t;
        uint64_t T_cur = st.T;
        const uint64_t j_cur = st.j, r_word = st.R;
        const int cur = st.cur, nxt = cur ^ 1;
        const R* const xb = (const R*)(cur ? fd.x[1] : fd.x[0]);
        const double* const tb = cur ? fd.theta[1] : fd.theta[0];
        keep_loaded(j_cur, cur, xb, tb, ztag);
        const uint64_t step = j_cur + 1;
        const bool ahead = ztag == step;   // this step's normals were drawn ahead
        const R* const zb = (const R*)fd.z;
        // the slot's normals, when drawn ahead: loaded first, as they depend
        // on nothing the search below finds (the innovation's only where they
        // are few enough to hold through the integration)
        R z[P];
        R zi[D];
        if (ahead && valid) {
#pragma unroll
            for (int i = 0; i < P; ++i) z[i] = zb[(size_t)i * fd.npad + n];
            if constexpr (D <= 4) {
#pragma unroll
                for (int i = 0; i < D; ++i) zi[i] = zb[(size_t)(P + i) * fd.npad + n];
            }
        }
        if constexpr (INL) {
            if (fold) {
                // 3(b) here: the draw's total and offset, then this slot's ancestor
                T_cur = tile_offsets<FOLD_MAX_TILES>(fd, Poff, shu);
                if (!(rec.t_next > t_cur)) continue;   // the step does not run
                const uint64_t V = T_cur ? __umul64hi(r_word, T_cur) : 0;
                if (itm.tile == 0 && threadIdx.x == 0) {
                    st.T = T_cur;
                    st.V = V;
                }
                if (T_cur == 0) continue;
                const uint64_t N = (uint64_t)fd.n;
                const uint64_t u = (uint64_t)n * T_cur + V;
                const int s_t = valid ? offset_tile(Poff, fd.ntiles, N, u) : 0;
                // the tiles of the first and the last valid slot bound every
                // slot's (ancestors are nondecreasing in the slot)
                const int last = (fd.n - itm.tile * TILE < TILE ? fd.n - itm.tile * TILE : TILE) - 1;
                if (threadIdx.x == 0) lo_sh[0] = s_t;
                if (threadIdx.x == last) lo_sh[1] = s_t;
                __syncthreads();
                const int s_a = lo_sh[0], s_b = lo_sh[1];
                if (s_b - s_a < FOLD_STAGE) {
                    for (int k = threadIdx.x; k < (s_b - s_a + 1) * TILE; k += TILE)
                        cqs[k] = fd.q[(size_t)s_a * TILE + k];
                    __syncthreads();
                    if (valid) k_anc = s_t * TILE + intile_lds(cqs + (s_t - s_a) * TILE, Poff[s_t], N, u);
                } else if (valid) {
                    k_anc = s_t * TILE + intile_global(fd.q + (size_t)s_t * TILE, Poff[s_t], N, u);
                }
                if (valid) fd.anc[n] = k_anc;
            }
        }
        if (!(rec.t_next > t_cur) || T_cur == 0) continue;
        const double h = (rec.t_next - t_cur) / fd.substeps;
        double l = -INFINITY;
        double th[P];
        R x[D];
#pragma unroll
        for (int i = 0; i < P; ++i) th[i] = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) x[i] = R(0);
        uint32_t iters = 0, fails = 0, nonf = 0;
        bool neg = false;
        if (valid) {
            int k = k_anc;
            // the scatter covers every slot exactly once; an out-of-range
            // ancestor would be a bug: keep the read in bounds, zero the weight
            const bool bad = k < 0 || k >= fd.n;
            if (bad) k = 0;
            // 3(c): the slot takes its ancestor's x_j, shrunk parameters and
            // predictor likelihood
#pragma unroll
            for (int i = 0; i < D; ++i) x[i] = xb[(size_t)i * fd.npad + k];
            double ta[P];
#pragma unroll
            for (int i = 0; i < P; ++i) ta[i] = tb[(size_t)i * fd.npad + k];
            const double lb = fd.lbar[k];
            // 4(a): theta_{j+1} = m + s L z (normals in the propagation precision)
            if (!ahead) {
                // the ancestor's loads are in flight while the normals are
                // drawn: keep the scheduler from sinking them below the generator
                __builtin_amdgcn_sched_barrier(0);
                normals<P, R>(fd.seed, step, (uint64_t)n, PUR_PROLIF, z);
            }
            const double a = fd.a;
            double m[P];
#pragma unroll
            for (int i = 0; i < P; ++i) m[i] = a * ta[i] + (1.0 - a) * st.theta_bar[i];
#pragma unroll
            for (int i = 0; i < P; ++i) {
                double v = 0.0;
#pragma unroll
                for (int c = 0; c <= i; ++c) v += st.L[i * fd.p + c] * (double)z[c];
                th[i] = m[i] + fd.s * v;
            }
            // 4(b)-(d): Psi with the local-error variance, then the innovation
            Model md;
            md.set_params(th, fd);
            R gam[D];
            R xw[D];
#pragma unroll
            for (int i = 0; i < D; ++i) xw[i] = x[i];
            const R* fl = sizeof(R) == 4 ? (const R*)fd.floor_f : (const R*)fd.floor_;
            integrate_lmm<Model, R, KORD, true, LMM>(md, xw, gam, h, fd.substeps, (R)fd.rtol, fl, fd.kmax, iters,
                                                     fails);
            if (!ahead) {
                normals<D, R>(fd.seed, step, (uint64_t)n, PUR_INNOV, zi);
            } else if constexpr (D > 4) {
#pragma unroll
                for (int i = 0; i < D; ++i) zi[i] = zb[(size_t)(P + i) * fd.npad + n];
            }
            R* xo = (R*)fd.x[nxt];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                x[i] = xw[i] + sqrt(gam[i]) * zi[i];
                xo[(size_t)i * fd.npad + n] = x[i];
                neg |= x[i] < R(0);
            }
#pragma unroll
            for (int i = 0; i < P; ++i) fd.theta[nxt][(size_t)i * fd.npad + n] = th[i];
            // 5: w = pi(y | x_{j+1}) / pi(y | xbar)
            l = loglik<R>(x, fd.obs, rec.y, rec.sigma, fd.m) - lb;
            if (!(l > -INFINITY) || bad) { l = -INFINITY; nonf = 1; }
            fd.logw[nxt][n] = l;
        }
        // 6 (partials): tile moments with shift theta_bar_j
        tile_moments<R, P, D>(l, valid, th, x, st.theta_bar, pack_counts(iters, fails, nonf),
                              fd.part1 + (size_t)2 * fd.ntiles + itm.tile, fd.part2 + itm.tile, fd.ntiles, sh, neg);
    }
}

}  // namespace pf

// the advection-diffusion model's kernels (they use the reductions, the tile
// partials and the step checks above; the moment pass below uses theirs)
#include "pf_advdiff.hip"

namespace pf {

// ---------------------------------------------------------------------------
// step 6: one workgroup per batch entry -- mean, covariance, ESS, Cholesky,
// commit, and the step's status by ticket (device ring and host-mapped ring)
// ---------------------------------------------------------------------------
// A step whose update did not run (all first-stage weights zero): its
// predictor counters, from the first-stage partials.
__device__ inline void add_predict_counts(const FilterDesc& fd, FilterState& st, double* sh)
{
    double ci = 0.0, cf = 0.0;
    for (int t = threadIdx.x; t < fd.ntiles; t += TILE) {
        ci += fd.part1[(size_t)2 * fd.ntiles + t];
        cf += fd.part1[(size_t)3 * fd.ntiles + t];
    }
    ci = block_sum(ci, sh);
    cf = block_sum(cf, sh);
    if (threadIdx.x == 0) {
        st.newton_pred += (unsigned long long)ci;
        st.newton_fails += (unsigned long long)cf;
    }
}

template <int P, int D>
__device__ __forceinline__ int32_t moment_step(const FilterDesc& fd, FilterState& st, const StepRec& rec, double* sh,
                                               double* tot)
{
    const MomPre pre = mom_prefetch<P>(st);
    moments_combine<P, D>(fd, tot, sh);   // reads only: runs ahead of the checks
    if (!(rec.t_next > pre.t)) return ST_EORDER;
    if (pre.T == 0) {
        add_predict_counts(fd, st, sh);
        return ST_EDEGENERATE;
    }
    if (threadIdx.x == 0) {
        st.step = pre.j + 1;
        st.t_next = rec.t_next;
    }
    return moments_finish<P, D>(fd, tot, pre, st, true, rec.t_next);
}

// advection-diffusion: the parameter moments as for the other models, then
// (committed steps) the weighted state mean from the per-tile state sums
__device__ __forceinline__ int32_t ad_moment_step(const FilterDesc& fd, FilterState& st, const StepRec& rec,
                                                  double* sh, double* tot)
{
    const int32_t s = moment_step<AD_P, 0>(fd, st, rec, sh, tot);
    if (s == ST_OK) ad_state_mean(fd, sh);
    return s;
}

// MDL: the model of every filter in the launch (MODEL_ROBERTSON,
// MODEL_CHAIN16 or MODEL_ADVDIFF), or 0 when the batch mixes models (chosen
// per filter); a single-model instance carries only that model's combine and
// tail.
template <bool INL, int MDL>
__global__ __launch_bounds__(TILE) void k_moments(Batch B, const FilterDesc* descs, FilterState* states,
                                                  int32_t* host_ring)
{
    __shared__ double sh[TILE];
    __shared__ double tot[NACC_MAX];
    // the inline form has one entry: workgroup 0 does its moments, without a
    // loop (nothing per-filter is hoisted and kept live across iterations);
    // for a kinetic model the other workgroups draw the normals of the step
    // after this one (this step's index is recorded by the count pass; if
    // this step does not commit, the tags do not match the next step and
    // its update kernel draws them itself)
    if constexpr (INL && (MDL == MODEL_ROBERTSON || MDL == MODEL_CHAIN16)) {
        if (blockIdx.x > 0) {
            const FilterDesc& fd = B.fd;
            const uint64_t next = states[uniform(B.one.slot)].j_run + 1;
            if constexpr (MDL == MODEL_ROBERTSON) draw_ahead<Robertson<double>>(fd, next, 1);
            else draw_ahead<Chain16<double>>(fd, next, 1);
            return;
        }
    }
    const int b_end = INL ? 1 : B.count;
    for (int b = blockIdx.x; b < b_end; b += INL ? b_end : gridDim.x) {   // inline: b = 0 only
        const StepRec rec = record<INL>(B, b);
        const int slot = uniform(rec.slot);
        const FilterDesc& fd = desc_of<INL>(B, descs, slot);
        FilterState& st = states[slot];
        using RB = Robertson<double>;
        using CH = Chain16<double>;
        int32_t status;
        if constexpr (MDL == MODEL_ROBERTSON) status = moment_step<RB::P, RB::D>(fd, st, rec, sh, tot);
        else if constexpr (MDL == MODEL_CHAIN16) status = moment_step<CH::P, CH::D>(fd, st, rec, sh, tot);
        else if constexpr (MDL == MODEL_ADVDIFF) status = ad_moment_step(fd, st, rec, sh, tot);
        else {
            const int model = uniform(fd.model);
            if (model == MODEL_ROBERTSON) status = moment_step<RB::P, RB::D>(fd, st, rec, sh, tot);
            else if (model == MODEL_CHAIN16) status = moment_step<CH::P, CH::D>(fd, st, rec, sh, tot);
            else status = ad_moment_step(fd, st, rec, sh, tot);
        }
        if (threadIdx.x == 0) {
            st.status = status;
            st.ring[rec.seq % RING] = status;
            host_ring[(size_t)slot * RING + rec.seq % RING] = status;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// test-only kernels
// ---------------------------------------------------------------------------
__global__ void k_test_philox(uint64_t n, const uint64_t* ctr, const uint64_t* key, uint64_t* out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t w[4];
    Philox::block(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key[2 * i],
                  key[2 * i + 1], w);
    for (int s = 0; s < 4; ++s) out[4 * i + s] = w[s];
}

template <int COUNT>
__global__ void k_test_normals(uint64_t n, uint64_t seed, uint64_t step, uint64_t purpose, double* out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double z[COUNT];
    normals<COUNT>(seed, step, i, purpose, z);
    for (int s = 0; s < COUNT; ++s) out[i * COUNT + s] = z[s];
}

template <class Model, class R, int KORD, bool LTE, int LMM>
__global__ __launch_bounds__(TILE) void k_test_propagate(const FilterDesc* fdp, uint64_t n, const double* xin,
                                                         const double* theta, double h, double* xout,
                                                         double* gamma, unsigned long long* iters_out)
{
    constexpr int D = Model::D, P = Model::P;
    __shared__ unsigned long long shu[NWAVE];
    const FilterDesc& fd = *fdp;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t iters = 0, fails = 0;
    if (i < n) {
        R x[D], gam[D];
        double th[P];
        for (int c = 0; c < D; ++c) x[c] = (R)xin[c * n + i];
        for (int c = 0; c < P; ++c) th[c] = theta[c * n + i];
        Model md;
        md.set_params(th, fd);
        const R* fl = sizeof(R) == 4 ? (const R*)fd.floor_f : (const R*)fd.floor_;
        integrate_lmm<Model, R, KORD, LTE, LMM>(md, x, gam, h, fd.substeps, (R)fd.rtol, fl, fd.kmax, iters,
                                                fails);
        for (int c = 0; c < D; ++c) {
            xout[c * n + i] = (double)x[c];
            if (LTE && gamma) gamma[c * n + i] = (double)gam[c];
        }
    }
    const unsigned long long s = block_sum_u64(iters, shu);
    if (threadIdx.x == 0 && iters_out) atomicAdd(iters_out, s);
}

}  // namespace pf

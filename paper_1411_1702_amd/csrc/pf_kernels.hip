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

// exclusive prefix sum over the block (uint64, exact); returns the total
__device__ inline unsigned long long block_exscan_u64(unsigned long long v, unsigned long long& excl,
                                                      unsigned long long* sh)
{
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    unsigned long long incl = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const unsigned long long t = __shfl_up(incl, o);
        if (l >= o) incl += t;
    }
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

// Combine per-tile log-domain partials part[t*stride + 0] = tile max,
// part[t*stride + 1 + a] = sums scaled by exp(-tile max), a < nsum, in a
// fixed order: out[a] = sum_t exp(max_t - M) part[t][1+a].  The sum with
// index sq (a sum of squared weights) scales with exp(2 (max_t - M)).
// With an LDS staging buffer (buf, buf_len doubles), tiles are read in
// coalesced chunks; the order of the sums depends only on ntiles, stride and
// buf_len.  Returns M.
__device__ __forceinline__ double combine_tiles(const double* part, int stride, int ntiles, int nsum, double* out,
                                double* sh /* >= TILE doubles */, int sq = -1, double* buf = nullptr,
                                int buf_len = 0)
{
    double mx = -INFINITY;
    for (int t = threadIdx.x; t < ntiles; t += TILE) mx = fmax(mx, part[(size_t)t * stride]);
    const double M = block_max(mx, sh);
    const int groups = TILE / nsum;
    const int a = threadIdx.x % nsum, g = threadIdx.x / nsum;
    double acc = 0.0;
    if (buf) {
        const int ch = buf_len / stride;
        for (int t0 = 0; t0 < ntiles; t0 += ch) {
            const int nt = min(ch, ntiles - t0);
            __syncthreads();
            const double* src = part + (size_t)t0 * stride;
            const int cnt = nt * stride;
            // issue all of this thread's loads before the first LDS store
            constexpr int PER = 32;
            for (int base = 0; base < cnt; base += PER * TILE) {
                double r[PER];
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int i = base + k * TILE + (int)threadIdx.x;
                    r[k] = i < cnt ? src[i] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int i = base + k * TILE + (int)threadIdx.x;
                    if (i < cnt) buf[i] = r[k];
                }
            }
            __syncthreads();
            // the tile max slot becomes the tile's scale factor
            for (int t = threadIdx.x; t < nt; t += TILE) {
                const double mt = buf[t * stride];
                buf[t * stride] = (mt > -INFINITY && M > -INFINITY) ? exp(mt - M) : 0.0;
            }
            __syncthreads();
            if (g < groups) {
                for (int t = g; t < nt; t += groups) {
                    const double sc = buf[t * stride];
                    acc += (a == sq ? sc * sc : sc) * buf[t * stride + 1 + a];
                }
            }
        }
    } else if (g < groups && M > -INFINITY) {
        for (int t = g; t < ntiles; t += groups) {
            const double mt = part[(size_t)t * stride];
            if (mt > -INFINITY) {
                const double sc = exp(mt - M);
                acc += (a == sq ? sc * sc : sc) * part[(size_t)t * stride + 1 + a];
            }
        }
    }
    __syncthreads();
    if (g < groups) sh[g * nsum + a] = acc;
    __syncthreads();
    if (threadIdx.x < nsum) {
        double s = 0.0;
        for (int gg = 0; gg < groups; ++gg) s += sh[gg * nsum + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
    return M;
}

// ---------------------------------------------------------------------------
// moments of the parameters for one tile: partial[0] = max l, then
// s0 = sum e, s00 = sum e^2, S1 = sum e d, S2 = sum e d d^T (upper triangle,
// row by row), Sx = sum e x, with e = exp(l - max) and d = theta - c.
// PM, DM bound p and d at compile time so every register index is static.
// ---------------------------------------------------------------------------
template <class R, int PM, int DM>
__device__ void tile_moments(double l, bool valid, const double* th, const R* x, const double* cshift,
                             int p, int d, double* out_part, double* sh)
{
    const double lv = valid ? l : -INFINITY;
    const double Mt = block_max(lv, sh);
    const double e = (valid && lv > -INFINITY) ? exp(lv - Mt) : 0.0;
    double dv[PM];
#pragma unroll
    for (int i = 0; i < PM; ++i) dv[i] = (i < p && e > 0.0) ? th[i] - cshift[i] : 0.0;
    __shared__ double wsum[NWAVE][NACC_MAX];
    const int w = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
    int a = 0;
    auto emit = [&](double v) {
        v = wave_sum(v);
        if (ln == 0) wsum[w][a] = v;
        ++a;
    };
    emit(e);
    emit(e * e);
#pragma unroll
    for (int i = 0; i < PM; ++i)
        if (i < p) emit(e * dv[i]);
#pragma unroll
    for (int i = 0; i < PM; ++i)
#pragma unroll
        for (int j = i; j < PM; ++j)
            if (j < p) emit(e * dv[i] * dv[j]);
#pragma unroll
    for (int i = 0; i < DM; ++i)
        if (i < d) emit(e > 0.0 ? e * (double)x[i] : 0.0);
    const int nsum = a;
    __syncthreads();
    if (threadIdx.x < nsum) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NWAVE; ++i) s += wsum[i][threadIdx.x];
        out_part[1 + threadIdx.x] = s;
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
template <int P, int D>
__device__ __forceinline__ void moments_tail(const double* tot, FilterState& st, bool flip)
{
    constexpr int NT = P * (P + 1) / 2;
    const double s0 = tot[0], s00 = tot[1];
    if (!(s0 > 0.0) || !isfinite(s0)) {
        st.status = ST_EDEGENERATE;
        return;
    }
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
    if (jit < 0) {
        st.status = ST_EDEGENERATE;
        return;
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            st.C[i * P + j] = cov(i, j);
            st.L[i * P + j] = j <= i ? L[i * (i + 1) / 2 + j] : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < P; ++i) st.theta_bar[i] += dm[i];
#pragma unroll
    for (int i = 0; i < D; ++i) st.state_mean[i] = tot[2 + P + NT + i] * inv;
    st.ess = s0 * s0 / s00;
    st.jitters += (unsigned long long)jit;
    if (flip) {
        st.cur ^= 1;
        st.j = st.step;
        st.t = st.t_next;
    }
    st.status = ST_OK;
}

constexpr int STAGE_LEN = 8192;   // doubles of LDS staging for the tile combine

__device__ __forceinline__ void finalize_moments(const FilterDesc& fd, FilterState& st, bool flip, double* sh,
                                                 double* buf)
{
    __shared__ double tot[NACC_MAX];
    combine_tiles(fd.part2, fd.nacc, fd.ntiles, fd.nacc - 1, tot, sh, 1, buf, STAGE_LEN);
    if (threadIdx.x == 0) {
        if (fd.p == 3 && fd.d == 3) moments_tail<3, 3>(tot, st, flip);
        else moments_tail<PMAX, DMAX>(tot, st, flip);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// common item decode and step validity
// ---------------------------------------------------------------------------
struct Item {
    int b, slot, tile;
};
// items, batch entries and slots are uniform over the workgroup; saying so
// lets the compiler use scalar loads for every descriptor field
__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline Item decode(uint32_t it, const StepRec* recs)
{
    Item r;
    it = (uint32_t)uniform((int)it);
    r.b = (int)(it >> 16);
    r.slot = uniform(recs[r.b].slot);
    r.tile = (int)(it & 0xFFFFu);
    return r;
}

// The step of batch entry b may run: its observation time is after the
// filter's current time (checked again, identically, by every kernel; the
// final kernel reports PF_EORDER).
__device__ inline bool step_valid(const StepRec& r, const FilterState& st) { return r.t_next > st.t; }

// ---------------------------------------------------------------------------
// step 1: prior draw and initial moment partials
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(TILE) void k_init(int slot, const FilterDesc* descs, FilterState* states)
{
    __shared__ double sh[TILE];
    const FilterDesc& fd = descs[slot];
    for (int tile = blockIdx.x; tile < fd.ntiles; tile += gridDim.x) {
        const int n = tile * TILE + threadIdx.x;
        const bool valid = n < fd.n;
        double th[PMAX];
        R xs[DMAX];
        for (int i = 0; i < PMAX; ++i) th[i] = 0.0;
        for (int i = 0; i < DMAX; ++i) xs[i] = R(0);
        if (valid) {
            double z[PMAX];
            normals<PMAX>(fd.seed, 0, (uint64_t)n, PUR_PRIOR, z);
            for (int i = 0; i < fd.p; ++i) {
                th[i] = fd.prior_mean[i] + fd.prior_sd[i] * z[i];
                fd.theta[0][(size_t)i * fd.npad + n] = th[i];
            }
            R* x = (R*)fd.x[0];
            for (int i = 0; i < fd.d; ++i) {
                xs[i] = (R)fd.x0[i];
                x[(size_t)i * fd.npad + n] = xs[i];
            }
            fd.logw[0][n] = -log((double)fd.n);
        }
        tile_moments<R, PMAX, DMAX>(-log((double)fd.n), valid, th, xs, fd.prior_mean, fd.p, fd.d,
                                    fd.part2 + (size_t)tile * fd.nacc, sh);
    }
}

// one workgroup: moments of the prior draw (the shift is the prior mean, which
// the host stored as theta_bar)
__global__ __launch_bounds__(TILE) void k_init_moments(int slot, const FilterDesc* descs, FilterState* states)
{
    __shared__ double sh[TILE];
    __shared__ double buf[STAGE_LEN];
    finalize_moments(descs[slot], states[slot], false, sh, buf);
}

// ---------------------------------------------------------------------------
// steps 2 and 3(a): shrink, predictor, first-stage log-weights
// ---------------------------------------------------------------------------
template <class Model, class R, int KORD>
__global__ __launch_bounds__(TILE) void k_predict(const uint32_t* items, int n_items, const StepRec* recs,
                                                  const FilterDesc* descs, FilterState* states)
{
    constexpr int D = Model::D, P = Model::P;
    __shared__ double sh[TILE];
    __shared__ unsigned long long shu[NWAVE];
    for (int itx = blockIdx.x; itx < n_items; itx += gridDim.x) {
        const Item itm = decode(items[itx], recs);
        const StepRec& rec = recs[itm.b];
        const FilterDesc& fd = descs[itm.slot];
        FilterState& st = states[itm.slot];
        if (!step_valid(rec, st)) continue;
        const double h = (rec.t_next - st.t) / fd.substeps;
        const int n = itm.tile * TILE + threadIdx.x;
        const bool valid = n < fd.n;
        const int cur = st.cur;
        double lg = -INFINITY;
        uint32_t iters = 0, fails = 0;
        if (valid) {
            const R* xb = (const R*)fd.x[cur];
            R x[D];
#pragma unroll
            for (int i = 0; i < D; ++i) x[i] = xb[(size_t)i * fd.npad + n];
            double m[P];
            const double a = fd.a;
#pragma unroll
            for (int i = 0; i < P; ++i)
                m[i] = a * fd.theta[cur][(size_t)i * fd.npad + n] + (1.0 - a) * st.theta_bar[i];
            Model md;
            md.set_params(m, fd);
            const R* fl = sizeof(R) == 4 ? (const R*)fd.floor_f : (const R*)fd.floor_;
            integrate<Model, R, KORD, false>(md, x, nullptr, h, fd.substeps, (R)fd.rtol, fl, fd.kmax,
                                             iters, fails);
            const double lb = loglik<R>(x, fd.obs, rec.y, rec.sigma, fd.m);
            lg = fd.logw[cur][n] + lb;
            if (!(lg > -INFINITY)) lg = -INFINITY;   // NaN -> zero weight
            fd.lbar[n] = lb;
            fd.lg[n] = lg;
        }
        const double Mt = block_max(lg, sh);
        const double e = lg > -INFINITY ? exp(lg - Mt) : 0.0;
        const double s = block_sum(e, sh);
        const unsigned long long it_sum = block_sum_u64(iters, shu);
        const unsigned long long fl_sum = block_sum_u64(fails, shu);
        if (threadIdx.x == 0) {
            fd.part1[2 * itm.tile] = Mt;
            fd.part1[2 * itm.tile + 1] = s;
            atomicAdd(&st.newton_pred, it_sum);
            if (fl_sum) atomicAdd(&st.newton_fails, fl_sum);
        }
    }
}

// ---------------------------------------------------------------------------
// step 3(b): systematic resampling in integers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_count(const uint32_t* items, int n_items, const StepRec* recs,
                                                const FilterDesc* descs, FilterState* states)
{
    __shared__ double sh[TILE];
    __shared__ double tot[1];
    __shared__ unsigned long long shu[NWAVE];
    for (int itx = blockIdx.x; itx < n_items; itx += gridDim.x) {
        const Item itm = decode(items[itx], recs);
        const FilterDesc& fd = descs[itm.slot];
        const FilterState& st = states[itm.slot];
        if (!fd.g_direct && !step_valid(recs[itm.b], st)) continue;
        double M = 0.0, S = 1.0;
        if (!fd.g_direct) {
            // the filter's first-stage log-sum-exp, from the tile partials
            M = combine_tiles(fd.part1, 2, fd.ntiles, 1, tot, sh);
            S = tot[0];
        }
        const bool ok = fd.g_direct || (M > -INFINITY && isfinite(M) && S > 0.0);
        const int n = itm.tile * TILE + threadIdx.x;
        unsigned long long q = 0;
        if (n < fd.n) {
            const double l = fd.lg[n];
            const double g = fd.g_direct ? l : (ok && l > -INFINITY ? exp(l - M) / S : 0.0);
            if (g > 0.0) q = (unsigned long long)floor(ldexp(g, fd.shift));
            fd.q[n] = q;
        }
        const unsigned long long ts = block_sum_u64(q, shu);
        if (threadIdx.x == 0) fd.tsum[itm.tile] = ts;
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

__global__ __launch_bounds__(TILE) void k_scatter(const uint32_t* items, int n_items, const StepRec* recs,
                                                  const FilterDesc* descs, FilterState* states)
{
    __shared__ unsigned long long shu[NWAVE];
    __shared__ int n_long;
    __shared__ uint32_t run_lo[TILE], run_hi[TILE];
    __shared__ int run_k[TILE];
    for (int itx = blockIdx.x; itx < n_items; itx += gridDim.x) {
        const Item itm = decode(items[itx], recs);
        const FilterDesc& fd = descs[itm.slot];
        FilterState& st = states[itm.slot];
        if (!fd.g_direct && !step_valid(recs[itm.b], st)) continue;
        // exclusive offset of this tile and total T of the integer weights
        unsigned long long pre = 0, all = 0;
        for (int t = threadIdx.x; t < fd.ntiles; t += TILE) {
            const unsigned long long v = fd.tsum[t];
            all += v;
            if (t < itm.tile) pre += v;
        }
        pre = block_sum_u64(pre, shu);
        const unsigned long long T = block_sum_u64(all, shu);
        uint64_t r;
        if (fd.g_direct) {
            r = st.V;   // test mode: the uniform word was stored by the host
        } else {
            uint64_t w[4];
            Philox::block(st.j + 1, 0, PUR_RESAMPLE, 0, fd.seed, 0, w);
            r = w[0];
        }
        const uint64_t V = T ? __umul64hi(r, T) : 0;
        if (itm.tile == 0 && threadIdx.x == 0) {
            st.T = T;
            if (!fd.g_direct) st.V = V;
        }
        if (T == 0) continue;
        const int n = itm.tile * TILE + threadIdx.x;
        const unsigned long long q = n < fd.n ? fd.q[n] : 0ull;
        unsigned long long ex;
        block_exscan_u64(q, ex, shu);
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

// ---------------------------------------------------------------------------
// steps 3(c)-5 per output slot
// ---------------------------------------------------------------------------
template <class Model, class R, int KORD>
__global__ __launch_bounds__(TILE) void k_update(const uint32_t* items, int n_items, const StepRec* recs,
                                                 const FilterDesc* descs, FilterState* states)
{
    constexpr int D = Model::D, P = Model::P;
    __shared__ double sh[TILE];
    __shared__ unsigned long long shu[NWAVE];
    for (int itx = blockIdx.x; itx < n_items; itx += gridDim.x) {
        const Item itm = decode(items[itx], recs);
        const StepRec& rec = recs[itm.b];
        const FilterDesc& fd = descs[itm.slot];
        FilterState& st = states[itm.slot];
        if (!step_valid(rec, st) || st.T == 0) continue;
        const double h = (rec.t_next - st.t) / fd.substeps;
        const uint64_t step = st.j + 1;
        const int n = itm.tile * TILE + threadIdx.x;
        const bool valid = n < fd.n;
        const int cur = st.cur, nxt = cur ^ 1;
        double l = -INFINITY;
        double th[PMAX];
        R x[DMAX];
#pragma unroll
        for (int i = 0; i < PMAX; ++i) th[i] = 0.0;
#pragma unroll
        for (int i = 0; i < DMAX; ++i) x[i] = R(0);
        uint32_t iters = 0, fails = 0, nonf = 0;
        if (valid) {
            int k = fd.anc[n];
            // the scatter covers every slot exactly once; an out-of-range
            // ancestor would be a bug: keep the read in bounds, zero the weight
            const bool bad = k < 0 || k >= fd.n;
            if (bad) k = 0;
            // 3(c): the slot takes its ancestor's x_j, shrunk parameters and
            // predictor likelihood
            const R* xb = (const R*)fd.x[cur];
#pragma unroll
            for (int i = 0; i < D; ++i) x[i] = xb[(size_t)i * fd.npad + k];
            const double a = fd.a;
            double m[P];
#pragma unroll
            for (int i = 0; i < P; ++i)
                m[i] = a * fd.theta[cur][(size_t)i * fd.npad + k] + (1.0 - a) * st.theta_bar[i];
            const double lb = fd.lbar[k];
            // 4(a): theta_{j+1} = m + s L z (normals in the propagation precision)
            R z[P];
            normals<P, R>(fd.seed, step, (uint64_t)n, PUR_PROLIF, z);
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
            integrate<Model, R, KORD, true>(md, xw, gam, h, fd.substeps, (R)fd.rtol, fl, fd.kmax, iters, fails);
            R zi[D];
            normals<D, R>(fd.seed, step, (uint64_t)n, PUR_INNOV, zi);
            R* xo = (R*)fd.x[nxt];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                x[i] = xw[i] + sqrt(gam[i]) * zi[i];
                xo[(size_t)i * fd.npad + n] = x[i];
            }
#pragma unroll
            for (int i = 0; i < P; ++i) fd.theta[nxt][(size_t)i * fd.npad + n] = th[i];
            // 5: w = pi(y | x_{j+1}) / pi(y | xbar)
            l = loglik<R>(x, fd.obs, rec.y, rec.sigma, fd.m) - lb;
            if (!(l > -INFINITY) || bad) { l = -INFINITY; nonf = 1; }
            fd.logw[nxt][n] = l;
        }
        const unsigned long long it_sum = block_sum_u64(iters, shu);
        const unsigned long long fl_sum = block_sum_u64(fails, shu);
        const unsigned long long nf_sum = block_sum_u64(nonf, shu);
        if (threadIdx.x == 0) {
            atomicAdd(&st.newton_upd, it_sum);
            if (fl_sum) atomicAdd(&st.newton_fails, fl_sum);
            if (nf_sum) atomicAdd(&st.nonfinite, nf_sum);
        }
        // 6 (partials): tile moments with shift theta_bar_j
        tile_moments<R, P, D>(l, valid, th, x, st.theta_bar, P, D,
                              fd.part2 + (size_t)itm.tile * fd.nacc, sh);
    }
}

// ---------------------------------------------------------------------------
// step 6: one workgroup per batch entry -- mean, covariance, ESS, Cholesky,
// commit, and the step's status by ticket (device ring and host-mapped ring)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_moments(const StepRec* recs, int count, const FilterDesc* descs,
                                                  FilterState* states, int32_t* host_ring)
{
    __shared__ double sh[TILE];
    __shared__ double buf[STAGE_LEN];
    for (int b = blockIdx.x; b < count; b += gridDim.x) {
        const StepRec& rec = recs[b];
        const int slot = uniform(rec.slot);
        const FilterDesc& fd = descs[slot];
        FilterState& st = states[slot];
        int32_t status;
        if (!step_valid(rec, st)) {
            status = ST_EORDER;
        } else if (st.T == 0) {
            status = ST_EDEGENERATE;
        } else {
            if (threadIdx.x == 0) {
                st.step = st.j + 1;
                st.t_next = rec.t_next;
            }
            __syncthreads();
            finalize_moments(fd, st, true, sh, buf);
            status = st.status;
        }
        __syncthreads();
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

template <class Model, class R, int KORD, bool LTE>
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
        integrate<Model, R, KORD, LTE>(md, x, gam, h, fd.substeps, (R)fd.rtol, fl, fd.kmax, iters,
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

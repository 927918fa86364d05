// pf_advdiff.hip -- the 2D periodic advection-diffusion model of Sec. 4 on
// the GPU.
//
// The semi-discrete system dU/dt = L(theta) U of Sec. 4 has
//   L = -(k1^2 B1^T B1 + k1 k3 (B1^T B2 + B2^T B1) + (k2^2 + k3^2) B2^T B2)
//       + c1 B1 + c2 B2,   B1 = I (x) l, B2 = l (x) I,
// with l the periodic difference matrix (1 on the diagonal, -1 below it and
// in the corner) and the grid stacked x fastest, U[iy * nt + ix].  Every
// factor is circulant along its axis, so the 2D discrete Fourier modes
// exp(2 pi i (ky iy + kx ix) / nt) are eigenvectors of L with eigenvalues
//   lambda = -(k1^2 |mu_x|^2 + 2 k1 k3 Re(conj(mu_x) mu_y) + (k2^2 + k3^2) |mu_y|^2)
//            + c1 mu_x + c2 mu_y,   mu = 1 - exp(-2 pi i k / nt).
// An implicit LMM step on this linear system is therefore one complex
// division per mode: the Newton iteration of Algorithm 1 steps 2 and 4(d)
// converges in its first iteration to (I - h beta L)^{-1} psi, which is what
// is computed here, mode by mode, with the same restart ramp, comparison
// values, error constants and SDIRK start-up as the kinetic models.  The
// local-error estimate of step 4(b) is formed per mode, taken back to the
// grid by an inverse transform and squared there, once per step.
//
// Layout: one workgroup per particle; the particle's field, the row
// transform and the half spectrum (kx = 0 .. nt/2, the rest is the complex
// conjugate) live in LDS; each thread keeps a few modes' LMM history in
// registers and owns a few quads of grid points (their innovation normals
// are one Philox block each).  The state is stored particle-major
// ([npad][d]), so a particle's field is one contiguous read or write.
// The transforms are plain O(nt^3) sums (nt <= 39, no power-of-two sizes),
// with the twiddles cos, sin(2 pi t / nt) in LDS.
#pragma once

namespace pf {

template <class R>
struct Cx {
    R re, im;
};
template <class R> __device__ inline Cx<R> cx(R re, R im) { return Cx<R>{re, im}; }
template <class R> __device__ inline Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> __device__ inline Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> __device__ inline Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
template <class R> __device__ inline Cx<R> operator*(Cx<R> a, Cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> __device__ inline Cx<R> cinv(Cx<R> a)
{
    const R r = recip(a.re * a.re + a.im * a.im);
    return {a.re * r, -a.im * r};
}

// launch shapes: threads per particle and the largest grid side they cover
template <int WGS_, int NTB_>
struct AdShape {
    static constexpr int WGS = WGS_, NTB = NTB_;
    static constexpr int KXB = NTB / 2 + 1;
    static constexpr int MPT = (NTB * KXB + WGS - 1) / WGS;            // modes per thread
    static constexpr int QPT = ((NTB * NTB + 3) / 4 + WGS - 1) / WGS;  // point quads per thread
};
using AdSmall = AdShape<64, 22>;    // one wavefront per particle, nt <= 22
using AdLarge = AdShape<256, 39>;   // four wavefronts per particle, nt <= 39

// model constants for the moment passes (P parameters; the state mean has
// its own per-tile sums, so D = 0 in the moment partials)
struct AdTag {
    static constexpr int P = AD_P, D = 0;
};

template <class R>
struct AdLds {
    R *P, *Yr, *Yi, *Zr, *Zi, *tc, *ts;
};

// LDS bytes of one particle's workspace
__host__ __device__ inline size_t ad_lds_bytes(int nt, int rsize)
{
    const int hm = nt * (nt / 2 + 1);
    return (size_t)(nt * nt + 4 * hm + 2 * nt) * (size_t)rsize;
}

template <class R>
__device__ inline AdLds<R> ad_lds(R* b, int nt)
{
    const int hm = nt * (nt / 2 + 1);
    AdLds<R> L;
    L.P = b;
    L.Yr = L.P + nt * nt;
    L.Yi = L.Yr + hm;
    L.Zr = L.Yi + hm;
    L.Zi = L.Zr + hm;
    L.tc = L.Zi + hm;
    L.ts = L.tc + nt;
    return L;
}

template <class R, int WGS>
__device__ inline void ad_twiddles(const AdLds<R>& L, int nt)
{
    for (int t = threadIdx.x; t < nt; t += WGS) {
        double s, c;
        sincospi(2.0 * t / nt, &s, &c);
        L.tc[t] = (R)c;
        L.ts[t] = (R)s;
    }
}

// forward transform along x (real field -> half spectrum rows):
//   Y[iy][q] = sum_ix P[iy][ix] exp(-2 pi i q ix / nt)
template <class R, int WGS, int NTC>
__device__ inline void dft_rows_fwd(const AdLds<R>& L, int nt_rt, int kx_rt)
{
    const int nt = NTC > 0 ? NTC : nt_rt, kx = NTC > 0 ? NTC / 2 + 1 : kx_rt;
    for (int o = threadIdx.x; o < nt * kx; o += WGS) {
        const int iy = o / kx, q = o - iy * kx;
        const R* row = L.P + iy * nt;
        R sr = R(0), si = R(0);
        int t = 0;
#pragma unroll(NTC > 0 ? NTC : 1)
        for (int ix = 0; ix < nt; ++ix) {
            const R v = row[ix];
            sr += v * L.tc[t];
            si -= v * L.ts[t];
            t += q;
            if (t >= nt) t -= nt;
        }
        L.Yr[o] = sr;
        L.Yi[o] = si;
    }
}

// forward transform along y: Z[ky][q] = sum_iy Y[iy][q] exp(-2 pi i ky iy / nt)
template <class R, int WGS, int NTC>
__device__ inline void dft_cols_fwd(const AdLds<R>& L, int nt_rt, int kx_rt)
{
    const int nt = NTC > 0 ? NTC : nt_rt, kx = NTC > 0 ? NTC / 2 + 1 : kx_rt;
    for (int o = threadIdx.x; o < nt * kx; o += WGS) {
        const int ky = o / kx, q = o - ky * kx;
        R sr = R(0), si = R(0);
        int t = 0;
#pragma unroll(NTC > 0 ? NTC : 1)
        for (int iy = 0; iy < nt; ++iy) {
            const R yr = L.Yr[iy * kx + q], yi = L.Yi[iy * kx + q];
            const R c = L.tc[t], s = L.ts[t];
            sr += yr * c + yi * s;
            si += yi * c - yr * s;
            t += ky;
            if (t >= nt) t -= nt;
        }
        L.Zr[o] = sr;
        L.Zi[o] = si;
    }
}

// inverse transform along y: Y[iy][q] = sum_ky Z[ky][q] exp(+2 pi i ky iy / nt)
template <class R, int WGS, int NTC>
__device__ inline void dft_cols_inv(const AdLds<R>& L, int nt_rt, int kx_rt)
{
    const int nt = NTC > 0 ? NTC : nt_rt, kx = NTC > 0 ? NTC / 2 + 1 : kx_rt;
    for (int o = threadIdx.x; o < nt * kx; o += WGS) {
        const int iy = o / kx, q = o - iy * kx;
        R sr = R(0), si = R(0);
        int t = 0;
#pragma unroll(NTC > 0 ? NTC : 1)
        for (int ky = 0; ky < nt; ++ky) {
            const R zr = L.Zr[ky * kx + q], zi = L.Zi[ky * kx + q];
            const R c = L.tc[t], s = L.ts[t];
            sr += zr * c - zi * s;
            si += zi * c + zr * s;
            t += iy;
            if (t >= nt) t -= nt;
        }
        L.Yr[o] = sr;
        L.Yi[o] = si;
    }
}

// inverse transform along x back to the real field, with the 1/nt^2 of the
// inverse: P[iy][ix] = scale sum_q w_q Re(Y[iy][q] exp(+2 pi i q ix / nt)),
// w_q = 1 for q = 0 and (even nt) q = nt/2, else 2 (the conjugate half)
template <class R, int WGS, int NTC>
__device__ inline void dft_rows_inv(const AdLds<R>& L, int nt_rt, int kx_rt, R scale)
{
    const int nt = NTC > 0 ? NTC : nt_rt, kx = NTC > 0 ? NTC / 2 + 1 : kx_rt;
    for (int o = threadIdx.x; o < nt * nt; o += WGS) {
        const int iy = o / nt, ix = o - iy * nt;
        const R* yr = L.Yr + iy * kx;
        const R* yi = L.Yi + iy * kx;
        R s = yr[0];
        int t = ix;
        if (t >= nt) t -= nt;
#pragma unroll(NTC > 0 ? NTC / 2 : 1)
        for (int q = 1; q < kx; ++q) {
            const R w = 2 * q == nt ? R(1) : R(2);
            s += w * (yr[q] * L.tc[t] - yi[q] * L.ts[t]);
            t += ix;
            if (t >= nt) t -= nt;
        }
        L.P[o] = scale * s;
    }
}

// Psi on the field in L.P (the caller has written it and the twiddles and
// synchronised): M steps of size h, BDF of order `korder` with the restart
// ramp, or with the SDIRK start-up when `sd`.  Leaves x_M in L.P; with LTE,
// gq receives the innovation variance at the thread's point quads.
template <class R, class S, bool LTE, int NTC>
__device__ void ad_propagate(const AdLds<R>& L, int nt_rt, const double (&th)[AD_P], double h_d, int M, int korder,
                             bool sd, R (&gq)[S::QPT][4])
{
    const int nt = NTC > 0 ? NTC : nt_rt;
    const int kx = nt / 2 + 1, hm = nt * kx, d = nt * nt;
    // modes per thread: from the grid side when it is known at compile time
    constexpr int MPT = NTC > 0 ? (NTC * (NTC / 2 + 1) + S::WGS - 1) / S::WGS : S::MPT;
    const int tid = threadIdx.x;
    const R h = (R)h_d;
    const R scale = R(1) / (R)(nt * nt);
    if constexpr (LTE) {
#pragma unroll
        for (int v = 0; v < S::QPT; ++v)
#pragma unroll
            for (int s = 0; s < 4; ++s) gq[v][s] = R(0);
    }
    dft_rows_fwd<R, S::WGS, NTC>(L, nt, kx);
    __syncthreads();
    dft_cols_fwd<R, S::WGS, NTC>(L, nt, kx);
    __syncthreads();
    // the thread's modes: eigenvalue and history x_{m-1} .. x_{m-4}
    const R k1 = (R)th[0], k2 = (R)th[1], k3 = (R)th[2], c1 = (R)th[3], c2 = (R)th[4];
    Cx<R> lam[MPT], h0[MPT], h1[MPT], h2[MPT], h3[MPT];
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
        const int j = tid + S::WGS * u;
        const int jj = j < hm ? j : 0;
        const int ky = jj / kx, q = jj - ky * kx;
        const Cx<R> mx = cx(R(1) - L.tc[q], L.ts[q]);
        const Cx<R> my = cx(R(1) - L.tc[ky], L.ts[ky]);
        const R ax = mx.re * mx.re + mx.im * mx.im, ay = my.re * my.re + my.im * my.im;
        const R cr = mx.re * my.re + mx.im * my.im;   // Re(conj(mu_x) mu_y)
        lam[u] = cx(-(k1 * k1 * ax + R(2) * k1 * k3 * cr + (k2 * k2 + k3 * k3) * ay) + c1 * mx.re + c2 * my.re,
                     c1 * mx.im + c2 * my.im);
        h0[u] = cx(L.Zr[jj], L.Zi[jj]);
        h1[u] = h2[u] = h3[u] = cx(R(0), R(0));
    }
    int avail = 0;
    for (int m = 1; m <= M; ++m) {
        const int q = avail < 1 ? 1 : (avail < korder ? avail : korder);
        const BdfCoef co = bdf_coef(q);
        const R c = h * (R)co.beta;
        const bool start = sd && korder >= 2 && avail < korder - 1;
#pragma unroll
        for (int u = 0; u < MPT; ++u) {
            const Cx<R> one = cx(R(1), R(0));
            const Cx<R> inv = cinv(one - c * lam[u]);
            Cx<R> xn;
            if (start) {
                // the SDIRK stages, mode by mode: Y = (x + h sum a_sj F_j) / (1 - h a_ss lambda)
                const Sdirk tb = korder == 2 ? sdirk_table<2>() : sdirk_table<3>();
                Cx<R> F[3];
                Cx<R> Y = h0[u];
#pragma unroll
                for (int sg = 0; sg < 3; ++sg) {
                    if (sg < korder) {
                        Cx<R> ps = h0[u];
#pragma unroll
                        for (int jn = 0; jn < sg; ++jn) ps = ps + (h * (R)tb.a[sg][jn]) * F[jn];
                        Y = ps * cinv(one - (h * (R)tb.a[sg][sg]) * lam[u]);
                        F[sg] = lam[u] * Y;
                    }
                }
                xn = Y;
            } else {
                const Cx<R> psi = (-(R)co.a1) * h0[u] - (R)co.a2 * h1[u] - (R)co.a3 * h2[u];
                xn = psi * inv;
            }
            if constexpr (LTE) {
                Cx<R> xp;
                if (avail == 0) xp = h0[u] + h * (lam[u] * h0[u]);
                else if (q == 1) xp = R(2) * h0[u] - h1[u];
                else if (q == 2) xp = R(3) * h0[u] - R(3) * h1[u] + h2[u];
                else xp = R(4) * h0[u] - R(6) * h1[u] + R(4) * h2[u] - h3[u];
                // the filtered Milne difference; at the first step, whose
                // comparison value is the Euler one, filtered twice
                const R kap = avail == 0 ? R(0.5) : (R)co.kappa;
                Cx<R> e = kap * ((xn - xp) * inv);
                if (avail == 0) e = e * inv;
                const int j = tid + S::WGS * u;
                if (j < hm) {
                    L.Zr[j] = e.re;
                    L.Zi[j] = e.im;
                }
            }
            h3[u] = h2[u];
            h2[u] = h1[u];
            h1[u] = h0[u];
            h0[u] = xn;
        }
        avail = avail < 3 ? avail + 1 : 3;
        if constexpr (LTE) {
            __syncthreads();
            dft_cols_inv<R, S::WGS, NTC>(L, nt, kx);
            __syncthreads();
            dft_rows_inv<R, S::WGS, NTC>(L, nt, kx, scale);
            __syncthreads();
#pragma unroll
            for (int v = 0; v < S::QPT; ++v)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int i = 4 * (tid + S::WGS * v) + s;
                    if (i < d) {
                        const R e = L.P[i];
                        gq[v][s] += e * e;
                    }
                }
        }
    }
    // x_M back on the grid
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
        const int j = tid + S::WGS * u;
        if (j < hm) {
            L.Zr[j] = h0[u].re;
            L.Zi[j] = h0[u].im;
        }
    }
    __syncthreads();
    dft_cols_inv<R, S::WGS, NTC>(L, nt, kx);
    __syncthreads();
    dft_rows_inv<R, S::WGS, NTC>(L, nt, kx, scale);
    __syncthreads();
}

// log pi(y | x) over the observed sites of the field in L.P, in the first
// wavefront (m <= 32); returned to every lane of that wavefront
template <class R>
__device__ inline double ad_loglik(const R* P, const FilterDesc& fd, const StepRec& rec)
{
    const int t = threadIdx.x;
    double s = 0.0;
    bool bad = false;
    if (t < fd.m) {
        const double v = (double)P[fd.obs[t]];
        bad = !isfinite(v);
        const double r = (rec.y[t] - v) / rec.sigma[t];
        s = r * r;
    }
    s = wave_sum(s);
    const bool anybad = __any(bad);
    return anybad ? -INFINITY : -0.5 * s;
}

// ---------------------------------------------------------------------------
// step 1: prior draw, the initial field, initial moment partials
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(TILE) void k_ad_init(int slot, const FilterDesc* descs, FilterState* states)
{
    __shared__ double sh[TILE];
    const FilterDesc& fd = descs[slot];
    const int d = fd.d;
    R* x = (R*)fd.x[0];
    for (int tile = blockIdx.x; tile < fd.ntiles; tile += gridDim.x) {
        const int n = tile * TILE + threadIdx.x;
        const bool valid = n < fd.n;
        double th[AD_P];
#pragma unroll
        for (int i = 0; i < AD_P; ++i) th[i] = 0.0;
        if (valid) {
            double z[AD_P];
            normals<AD_P>(fd.seed, 0, (uint64_t)n, PUR_PRIOR, z);
#pragma unroll
            for (int i = 0; i < AD_P; ++i) {
                th[i] = fd.prior_mean[i] + fd.prior_sd[i] * z[i];
                fd.theta[0][(size_t)i * fd.npad + n] = th[i];
            }
            fd.logw[0][n] = -log((double)fd.n);
        }
        // the tile's fields, contiguous: element e of the tile is (particle e / d, point e % d)
        const size_t base = (size_t)tile * TILE * d;
        for (int e = threadIdx.x; e < TILE * d; e += TILE) x[base + e] = (R)fd.x0b[e % d];
        tile_moments<R, AD_P, 0>(-log((double)fd.n), valid, th, nullptr, fd.prior_mean, 0, nullptr,
                                 fd.part2 + tile, fd.ntiles, sh);
    }
}

// ---------------------------------------------------------------------------
// steps 2 and 3(a): shrink, predictor, first-stage log-weights (one
// workgroup per particle), then the tile partials of the first stage
// ---------------------------------------------------------------------------
template <class R, class S, int NTC>
__global__ __launch_bounds__(S::WGS) void k_ad_predict(StepRec rec, int slot, const FilterDesc* descs,
                                                       FilterState* states)
{
    extern __shared__ double ad_smem[];
    const FilterDesc& fd = descs[slot];
    const FilterState& st = states[slot];
    if (!step_valid(rec, st)) return;
    const int nt = NTC > 0 ? NTC : fd.nt, d = nt * nt;
    const AdLds<R> L = ad_lds<R>((R*)ad_smem, nt);
    const double h = (rec.t_next - st.t) / fd.substeps;
    const int cur = st.cur;
    ad_twiddles<R, S::WGS>(L, nt);
    R gq[S::QPT][4];
    for (int n = blockIdx.x; n < fd.n; n += gridDim.x) {
        const R* xb = (const R*)fd.x[cur] + (size_t)n * d;
        for (int i = threadIdx.x; i < d; i += S::WGS) L.P[i] = xb[i];
        double m[AD_P];
#pragma unroll
        for (int i = 0; i < AD_P; ++i)
            m[i] = fd.a * fd.theta[cur][(size_t)i * fd.npad + n] + (1.0 - fd.a) * st.theta_bar[i];
        __syncthreads();
        ad_propagate<R, S, false, NTC>(L, nt, m, h, fd.substeps, fd.order, fd.lmm == 2, gq);
        if (threadIdx.x < WAVE) {
            const double lb = ad_loglik<R>(L.P, fd, rec);
            if (threadIdx.x == 0) {
                double lg = fd.logw[cur][n] + lb;
                if (!(lg > -INFINITY)) lg = -INFINITY;
                fd.lbar[n] = lb;
                fd.lg[n] = lg;
            }
        }
        __syncthreads();
    }
}

// tile partials of the first stage: (max, sum exp) of the log-weights, and
// the predictor's integration steps (one linear solve each)
__global__ __launch_bounds__(TILE) void k_ad_part1(StepRec rec, int slot, const FilterDesc* descs,
                                                   FilterState* states)
{
    __shared__ double sh[TILE];
    const FilterDesc& fd = descs[slot];
    const FilterState& st = states[slot];
    if (!step_valid(rec, st)) return;
    for (int tile = blockIdx.x; tile < fd.ntiles; tile += gridDim.x) {
        const int n = tile * TILE + threadIdx.x;
        const double lg = n < fd.n ? fd.lg[n] : -INFINITY;
        const double Mt = block_max(lg, sh);
        const double s = block_sum(lg > -INFINITY ? exp(lg - Mt) : 0.0, sh);
        if (threadIdx.x == 0) {
            const size_t cs = (size_t)fd.ntiles;
            const int cnt = min(TILE, fd.n - tile * TILE);
            fd.part1[tile] = Mt;
            fd.part1[cs + tile] = s;
            fd.part1[2 * cs + tile] = (double)cnt * fd.substeps;
            fd.part1[3 * cs + tile] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// steps 3(c), 4, 5: one workgroup per output slot
// ---------------------------------------------------------------------------
template <class R, class S, int NTC>
__global__ __launch_bounds__(S::WGS) void k_ad_update(StepRec rec, int slot, const FilterDesc* descs,
                                                      FilterState* states)
{
    extern __shared__ double ad_smem[];
    const FilterDesc& fd = descs[slot];
    const FilterState& st = states[slot];
    if (!step_valid(rec, st) || st.T == 0) return;
    const int nt = NTC > 0 ? NTC : fd.nt, d = nt * nt;
    const AdLds<R> L = ad_lds<R>((R*)ad_smem, nt);
    const double h = (rec.t_next - st.t) / fd.substeps;
    const uint64_t step = st.j + 1;
    const int cur = st.cur, nxt = cur ^ 1;
    const int tid = threadIdx.x;
    ad_twiddles<R, S::WGS>(L, nt);
    R gq[S::QPT][4];
    for (int n = blockIdx.x; n < fd.n; n += gridDim.x) {
        int k = fd.anc[n];
        // the scatter covers every slot exactly once; an out-of-range
        // ancestor would be a bug: keep the reads in bounds, zero the weight
        const bool bad = k < 0 || k >= fd.n;
        if (bad) k = 0;
        // 3(c): the ancestor's field, shrunk parameters, predictor likelihood
        const R* xb = (const R*)fd.x[cur] + (size_t)k * d;
        for (int i = tid; i < d; i += S::WGS) L.P[i] = xb[i];
        double th[AD_P];
        {
            double m[AD_P];
#pragma unroll
            for (int i = 0; i < AD_P; ++i)
                m[i] = fd.a * fd.theta[cur][(size_t)i * fd.npad + k] + (1.0 - fd.a) * st.theta_bar[i];
            // 4(a): theta_{j+1} = m + s L z
            R z[AD_P];
            normals<AD_P, R>(fd.seed, step, (uint64_t)n, PUR_PROLIF, z);
#pragma unroll
            for (int i = 0; i < AD_P; ++i) {
                double v = 0.0;
#pragma unroll
                for (int c = 0; c <= i; ++c) v += st.L[i * fd.p + c] * (double)z[c];
                th[i] = m[i] + fd.s * v;
            }
        }
        const double lb = fd.lbar[k];
        __syncthreads();
        // 4(b)-(d): Psi with the local-error variance, then the innovation
        ad_propagate<R, S, true, NTC>(L, nt, th, h, fd.substeps, fd.order, fd.lmm == 2, gq);
        R* xo = (R*)fd.x[nxt] + (size_t)n * d;
#pragma unroll
        for (int v = 0; v < S::QPT; ++v) {
            const int qd = tid + S::WGS * v;
            if (4 * qd < d) {
                uint64_t w[4];
                Philox::block(step, (uint64_t)n, PUR_INNOV, (uint64_t)qd, fd.seed, 0, w);
                R z[4];
                box_muller((R)unit_open(w[0]), (R)unit_open(w[1]), z[0], z[1]);
                box_muller((R)unit_open(w[2]), (R)unit_open(w[3]), z[2], z[3]);
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int i = 4 * qd + s;
                    if (i < d) {
                        const R xv = L.P[i] + sqrt(gq[v][s]) * z[s];
                        L.P[i] = xv;
                        xo[i] = xv;
                    }
                }
            }
        }
        __syncthreads();
        // 5: w = pi(y | x_{j+1}) / pi(y | xbar of the ancestor)
        if (tid < WAVE) {
            double l = ad_loglik<R>(L.P, fd, rec) - lb;
            if (tid == 0) {
                if (!(l > -INFINITY) || bad) l = -INFINITY;
                fd.logw[nxt][n] = l;
            }
            if (tid < AD_P) {
#pragma unroll
                for (int i = 0; i < AD_P; ++i)
                    if (tid == i) fd.theta[nxt][(size_t)i * fd.npad + n] = th[i];
            }
        }
        __syncthreads();
    }
}

// tile partials of step 6, one workgroup per (tile, chunk of 64 grid
// points): the weighted state sums of the chunk over the tile's particles,
// scaled by the tile's largest log-weight (each of the four wavefronts sums
// every fourth particle, then the four are added); chunk 0 also writes the
// parameter moments (tile_moments, shift theta_bar_j) and the counters (one
// linear solve per integration step).
constexpr int AD_CHUNK = 64;

template <class R>
__global__ __launch_bounds__(TILE) void k_ad_part2(StepRec rec, int slot, const FilterDesc* descs,
                                                   FilterState* states)
{
    __shared__ double sh[TILE];
    __shared__ double ew[TILE];
    __shared__ double red[NWAVE][AD_CHUNK];
    const FilterDesc& fd = descs[slot];
    const FilterState& st = states[slot];
    if (!step_valid(rec, st) || st.T == 0) return;
    const int nxt = st.cur ^ 1, d = fd.d;
    const int nch = (d + AD_CHUNK - 1) / AD_CHUNK;
    const R* x = (const R*)fd.x[nxt];
    for (int b = blockIdx.x; b < fd.ntiles * nch; b += gridDim.x) {
        const int tile = b / nch, chunk = b - tile * nch;
        const int n = tile * TILE + threadIdx.x;
        const bool valid = n < fd.n;
        const double l = valid ? fd.logw[nxt][n] : -INFINITY;
        if (chunk == 0) {
            double th[AD_P];
#pragma unroll
            for (int i = 0; i < AD_P; ++i) th[i] = valid ? fd.theta[nxt][(size_t)i * fd.npad + n] : 0.0;
            const uint32_t nonf = valid && !(l > -INFINITY) ? 1u : 0u;
            const uint64_t counts = pack_counts(valid ? (uint32_t)fd.substeps : 0u, 0u, nonf);
            tile_moments<R, AD_P, 0>(l, valid, th, nullptr, st.theta_bar, counts,
                                     fd.part1 + (size_t)2 * fd.ntiles + tile, fd.part2 + tile, fd.ntiles, sh);
        }
        const double Mt = block_max(l, sh);
        ew[threadIdx.x] = l > -INFINITY ? exp(l - Mt) : 0.0;
        __syncthreads();
        const int cnt = min(TILE, fd.n - tile * TILE);
        const int c = threadIdx.x % AD_CHUNK, g = threadIdx.x / AD_CHUNK;
        const int i = chunk * AD_CHUNK + c;
        double s = 0.0;
        if (i < d) {
            const R* xt = x + (size_t)tile * TILE * d + i;
            for (int r = g; r < cnt; r += NWAVE) {
                const double e = ew[r];
                if (e > 0.0) s += e * (double)xt[(size_t)r * d];
            }
        }
        red[g][c] = s;
        __syncthreads();
        if (g == 0 && i < d) {
            double t = red[0][c];
#pragma unroll
            for (int w = 1; w < NWAVE; ++w) t += red[w][c];
            fd.partx[(size_t)i * fd.ntiles + tile] = t;
        }
        __syncthreads();
    }
}

// the weighted state mean from the per-tile sums (after a committed step)
__device__ inline void ad_state_mean(const FilterDesc& fd, double* sh)
{
    const int nt = fd.ntiles;
    double mx = -INFINITY;
    for (int t = threadIdx.x; t < nt; t += TILE) mx = fmax(mx, fd.part2[t]);
    mx = block_max(mx, sh);
    double s0 = 0.0;
    for (int t = threadIdx.x; t < nt; t += TILE) {
        const double mt = fd.part2[t];
        if (mt > -INFINITY) s0 += exp(mt - mx) * fd.part2[(size_t)nt + t];
    }
    s0 = block_sum(s0, sh);
    const double inv = 1.0 / s0;
    for (int i = threadIdx.x; i < fd.d; i += TILE) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) {
            const double mt = fd.part2[t];
            if (mt > -INFINITY) s += exp(mt - mx) * fd.partx[(size_t)i * nt + t];
        }
        fd.smb[i] = s * inv;
    }
}

// ---------------------------------------------------------------------------
// test-only: Psi for n particles, x_in / x_out / gamma [d][n], theta [p][n]
// ---------------------------------------------------------------------------
template <class R, class S, bool LTE, int NTC>
__global__ __launch_bounds__(S::WGS) void k_ad_test_propagate(const FilterDesc* fdp, uint64_t n, const double* xin,
                                                              const double* theta, double h, double* xout,
                                                              double* gamma, unsigned long long* iters_out)
{
    extern __shared__ double ad_smem[];
    const FilterDesc& fd = *fdp;
    const int nt = NTC > 0 ? NTC : fd.nt, d = nt * nt;
    const AdLds<R> L = ad_lds<R>((R*)ad_smem, nt);
    const int tid = threadIdx.x;
    ad_twiddles<R, S::WGS>(L, nt);
    R gq[S::QPT][4];
    for (uint64_t p = blockIdx.x; p < n; p += gridDim.x) {
        for (int i = tid; i < d; i += S::WGS) L.P[i] = (R)xin[(size_t)i * n + p];
        double th[AD_P];
#pragma unroll
        for (int i = 0; i < AD_P; ++i) th[i] = theta[(size_t)i * n + p];
        __syncthreads();
        ad_propagate<R, S, LTE, NTC>(L, nt, th, h, fd.substeps, fd.order, fd.lmm == 2, gq);
        for (int i = tid; i < d; i += S::WGS) xout[(size_t)i * n + p] = (double)L.P[i];
        if (LTE && gamma) {
#pragma unroll
            for (int v = 0; v < S::QPT; ++v)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int i = 4 * (tid + S::WGS * v) + s;
                    if (i < d) gamma[(size_t)i * n + p] = (double)gq[v][s];
                }
        }
        if (tid == 0 && iters_out) atomicAdd(iters_out, (unsigned long long)fd.substeps);
        __syncthreads();
    }
}

}  // namespace pf

// pf_device.hpp -- per-lane device mathematics of the sampler: the
// counter-based RNG, the two models, and the BDF integrator Psi with its
// Newton solve and local-error estimate (Algorithm 1, steps 2 and 4).
// One particle per lane; everything here lives in registers.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf_types.hpp"

namespace pf {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies; the key advances by the Weyl constants between
// rounds.  Counter words are (step, particle, purpose, block), key (seed, 0).
// ---------------------------------------------------------------------------
struct Philox {
    static constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ULL;
    static constexpr uint64_t kMulB = 0xCA5A826395121157ULL;
    static constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ULL;
    static constexpr uint64_t kWeylB = 0xBB67AE8584CAA73BULL;

    // full 64x64 -> 128-bit product from four 32x32 -> 64 partial products
    // (each one multiply-add with a 64-bit addend), sharing the partial
    // products between the low and the high word
    __device__ static inline void mulhilo(uint64_t m, uint64_t a, uint64_t& lo, uint64_t& hi)
    {
        const uint32_t ml = (uint32_t)m, mh = (uint32_t)(m >> 32);
        const uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32);
        const uint64_t p0 = (uint64_t)ml * al;
        const uint64_t p1 = (uint64_t)mh * al + (p0 >> 32);
        const uint64_t p2 = (uint64_t)ml * ah + (uint32_t)p1;
        hi = (uint64_t)mh * ah + (p1 >> 32) + (p2 >> 32);
        lo = (p2 << 32) | (uint32_t)p0;
    }

    __device__ static inline void block(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                        uint64_t k0, uint64_t k1, uint64_t out[4])
    {
#pragma unroll
        for (int round = 0; round < 10; ++round) {
            uint64_t pa_lo, pa_hi, pb_lo, pb_hi;
            mulhilo(kMulA, c0, pa_lo, pa_hi);
            mulhilo(kMulB, c2, pb_lo, pb_hi);
            const uint64_t n0 = pb_hi ^ c1 ^ k0;
            const uint64_t n2 = pa_hi ^ c3 ^ k1;
            c0 = n0;
            c1 = pb_lo;
            c2 = n2;
            c3 = pa_lo;
            k0 += kWeylA;
            k1 += kWeylB;
        }
        out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
    }
};

// (0,1) uniform from the top 53 bits of a word
__device__ inline double unit_open(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1p-53; }

// Box-Muller pair from two uniforms, FP64 or FP32 (the innovation normals
// of FP32 propagation: the FP64 uniforms rounded to float).  The angle 2 pi u
// goes through sincospi of 2u, which is exact in binary, so the argument
// needs neither the rounded product by 2 pi nor a range reduction.
__device__ inline void box_muller(double u0, double u1, double& z0, double& z1)
{
    const double rad = sqrt(-2.0 * log(u0));
    double sn, cs;
    sincospi(2.0 * u1, &sn, &cs);
    z0 = rad * cs;
    z1 = rad * sn;
}
__device__ inline void box_muller(float u0, float u1, float& z0, float& z1)
{
    const float rad = sqrtf(-2.0f * logf(u0));
    float sn, cs;
    sincospif(2.0f * u1, &sn, &cs);
    z0 = rad * cs;
    z1 = rad * sn;
}

// `count` standard normals of one (step, particle, purpose): block b gives
// words w0..w3 and the Box-Muller pairs (w0, w1) and (w2, w3).
template <int COUNT, class RT = double>
__device__ inline void normals(uint64_t seed, uint64_t step, uint64_t particle, uint64_t purpose,
                               RT z[COUNT])
{
#pragma unroll
    for (int b = 0; b < (COUNT + 3) / 4; ++b) {
        uint64_t w[4];
        Philox::block(step, particle, purpose, (uint64_t)b, seed, 0, w);
        RT v[4];
        box_muller((RT)unit_open(w[0]), (RT)unit_open(w[1]), v[0], v[1]);
        box_muller((RT)unit_open(w[2]), (RT)unit_open(w[3]), v[2], v[3]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (4 * b + s < COUNT) z[4 * b + s] = v[s];
    }
}

// rate constant from a log-parameter, in the propagation precision: FP64
// exp for FP64 propagation; for FP32 propagation expf of the parameter
// rounded to FP32 (relative error of the rate about |theta| 2^-24, below the
// Newton tolerance of that path, at a third of the FP64 exp's instructions)
__device__ inline double exp_rate(double th, double) { return exp(th); }
__device__ inline float exp_rate(double th, float) { return expf((float)th); }

// fused multiply-add a b + c, one rounding
__device__ inline float rfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double rfma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// reciprocal: single-instruction v_rcp_f32 in FP32 (about 1 ulp); in FP64
// v_rcp_f64's estimate refined by two Newton-Raphson steps r += r (1 - v r),
// each of which squares the relative error (within about 1 ulp; the
// correctly rounded division takes twice the instructions).  Used where
// v is finite and nonzero (Newton pivots, K + x, |a|^2).
__device__ inline float recip(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ inline double recip(double v)
{
    double r = __builtin_amdgcn_rcp(v);
    r = __builtin_fma(r, __builtin_fma(-v, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-v, r, 1.0), r);
}

// |v| and max(a, b) as single instructions (max returns the non-NaN operand)
__device__ inline float rabs(float v) { return fabsf(v); }
__device__ inline double rabs(double v) { return fabs(v); }
__device__ inline float rmax(float a, float b) { return fmaxf(a, b); }
__device__ inline double rmax(double a, double b) { return fmax(a, b); }

// ---------------------------------------------------------------------------
// Models.  `eval` returns f(x) and the factorisation of the Newton matrix
// A = I - c J(x); `solve` overwrites b with A^{-1} b.
// ---------------------------------------------------------------------------

// Robertson kinetics.  The three rates move mass between the species, so
// f sums to zero, the columns of J sum to zero, and 1^T A = 1^T for
// A = I - cJ: the solution of A d = b has d1 + d2 + d3 = b1 + b2 + b3 = s
// for every b.  `solve` takes rows 2 and 3 of A with d1 = s - d2 - d3
// substituted,
//   (1 + c(k1 + 2 k2 x2 + k3 x3)) d2 + c(k1 + k3 x2) d3 = b2 + c k1 s
//   -2 c k2 x2 d2 + d3 = b3,
// and eliminates d3: the exact solution of the 3x3 system, with one
// reciprocal per factorisation.  For x >= 0 the pivot is >= 1.
template <class R>
struct Robertson {
    static constexpr int D = 3;
    static constexpr int P = 3;
    R k1, k2, k3;

    struct LU { R ck1, a12, t, inv; };

    __device__ inline void set_params(const double th[P], const FilterDesc&)
    {
        k1 = exp_rate(th[0], R(0));
        k2 = exp_rate(th[1], R(0));
        k3 = exp_rate(th[2], R(0));
    }

    // f alone (the Adams-Moulton history needs f at each accepted value)
    __device__ inline void rhs(const R x[D], R f[D]) const
    {
        const R r1 = k1 * x[0];
        const R r2 = k2 * x[1] * x[1];
        const R r3 = k3 * x[1] * x[2];
        f[0] = r3 - r1;
        f[1] = r1 - r2 - r3;
        f[2] = r2;
    }

    __device__ inline void eval(const R x[D], R c, R f[D], LU& lu) const
    {
        rhs(x, f);
        const R ck3 = c * k3;
        lu.ck1 = c * k1;
        lu.t = R(2) * c * k2 * x[1];                  // -A32
        const R a22 = (R(1) + lu.ck1) + lu.t + ck3 * x[2];
        lu.a12 = lu.ck1 + ck3 * x[1];
        lu.inv = recip(a22 + lu.a12 * lu.t);
    }

    __device__ inline void solve(const LU& lu, R b[D]) const
    {
        const R s = b[0] + b[1] + b[2];
        const R d2 = ((b[1] + lu.ck1 * s) - lu.a12 * b[2]) * lu.inv;
        const R d3 = b[2] + lu.t * d2;
        b[0] = s - d2 - d3;
        b[1] = d2;
        b[2] = d3;
    }
};

// 16-compartment chain with Michaelis-Menten losses,
//   x_i' = k_{i-1} x_{i-1} - k_i x_i - V_i x_i / (K_i + x_i),  unit influx at i = 1.
// J is lower bidiagonal, so A = I - cJ is solved by forward substitution.
template <class R>
struct Chain16 {
    static constexpr int D = 16;
    static constexpr int P = 12;
    R k[D];
    const R* VK;   // [V(16), K(16)], wave-uniform

    struct LU { R inv[D]; R c; };

    __device__ inline void set_params(const double th[P], const FilterDesc& fd)
    {
#pragma unroll
        for (int i = 0; i < D; ++i) k[i] = i < P ? exp_rate(th[i], R(0)) : (R)fd.rates_fixed[i];
        if constexpr (sizeof(R) == 4) VK = (const R*)fd.mc_f;
        else VK = (const R*)fd.mc;
    }

    __device__ inline void rhs(const R x[D], R f[D]) const
    {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const R V = VK[i], K = VK[D + i];
            const R inflow = i == 0 ? R(1) : k[i - 1] * x[i - 1];
            f[i] = inflow - k[i] * x[i] - V * x[i] * recip(K + x[i]);
        }
    }

    __device__ inline void eval(const R x[D], R c, R f[D], LU& lu) const
    {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const R V = VK[i], K = VK[D + i];
            const R r = recip(K + x[i]);
            const R inflow = i == 0 ? R(1) : k[i - 1] * x[i - 1];
            f[i] = inflow - k[i] * x[i] - V * x[i] * r;
            lu.inv[i] = recip(R(1) + c * (k[i] + V * K * r * r));
        }
        lu.c = c;
    }

    __device__ inline void solve(const LU& lu, R b[D]) const
    {
        b[0] = b[0] * lu.inv[0];
#pragma unroll
        for (int i = 1; i < D; ++i) b[i] = (b[i] + lu.c * k[i - 1] * b[i - 1]) * lu.inv[i];
    }
};

// ---------------------------------------------------------------------------
// Psi: M fixed BDF steps of size h from x (overwritten with the result).
// Step m uses order q = max(1, min(KORD, m-1)); the Newton iteration starts
// from x_{m-1} at m = 1 and from the degree-q extrapolation afterwards; stop
// when every |dx_i| <= rtol * max(|x_i|, floor_i), or after kmax iterations.
// With LTE, gam accumulates the squared filtered Milne estimates
//   e_m = kappa_q (I - h beta_q J)^{-1} (x_m - x_m^(0)),
// x^(0) being the extrapolation (kappa = |C|/(1+|C|)) or, at m = 1, the
// Euler value x_0 + h f(x_0) (kappa = 1/2); J from the last Newton iteration.
// At m = 1 the difference is solved with that matrix twice: the Euler value's
// error in a stiff mode is (1 - h lambda) times a stable predictor's, and the
// second solve brings the estimate to the order of the true local error.
// ---------------------------------------------------------------------------
struct BdfCoef {
    double a1, a2, a3;   // x_m + a1 x_{m-1} + a2 x_{m-2} + a3 x_{m-3} = h beta f_m
    double beta;
    double kappa;        // |C_{q+1}| / (1 + |C_{q+1}|)
};

__device__ inline BdfCoef bdf_coef(int q)
{
    if (q == 1) return {-1.0, 0.0, 0.0, 1.0, 1.0 / 3.0};
    if (q == 2) return {-4.0 / 3.0, 1.0 / 3.0, 0.0, 2.0 / 3.0, 2.0 / 11.0};
    return {-18.0 / 11.0, 9.0 / 11.0, -2.0 / 11.0, 6.0 / 11.0, 3.0 / 25.0};
}

// Start-up tables (SD): L-stable, stiffly accurate SDIRK of order KORD for the
// first KORD-1 steps of each interval (Alexander 1977): order 2 with
// gamma = 1 - 1/sqrt(2); order 3 with gamma the root of
// gamma^3 - 3 gamma^2 + 3 gamma/2 - 1/6 in (1/6, 1/2).
struct Sdirk {
    double a[3][3];
};
template <int K>
__device__ inline Sdirk sdirk_table()
{
    Sdirk t{};
    if constexpr (K == 2) {
        const double g = 0.29289321881345254;
        t.a[0][0] = g;
        t.a[1][0] = 1.0 - g;
        t.a[1][1] = g;
    } else {
        const double g = 0.43586652150845967;
        t.a[0][0] = g;
        t.a[1][0] = (1.0 - g) / 2.0;
        t.a[1][1] = g;
        t.a[2][0] = -(6.0 * g * g - 16.0 * g + 1.0) / 4.0;
        t.a[2][1] = (6.0 * g * g - 20.0 * g + 5.0) / 4.0;
        t.a[2][2] = g;
    }
    return t;
}

// one Newton solve of y = psi + c f(y) from the guess in y (the same
// iteration and stopping test as the BDF steps); the last factorisation is
// left in lu
template <class Model, class R>
__device__ inline void newton(const Model& md, R (&y)[Model::D], const R (&psi)[Model::D], R c, R rtol,
                              const R (&fl)[Model::D], int kmax, typename Model::LU& lu, uint32_t& iters,
                              uint32_t& fails)
{
    constexpr int D = Model::D;
    bool ok = false;
    int it = 0;
    do {
        R f[D];
        md.eval(y, c, f, lu);
        R b[D];
#pragma unroll
        for (int i = 0; i < D; ++i) b[i] = (psi[i] + c * f[i]) - y[i];
        md.solve(lu, b);
        ok = true;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            y[i] += b[i];
            ok &= rabs(b[i]) <= rtol * rmax(rabs(y[i]), fl[i]);
        }
        ++it;
    } while (!ok && it < kmax);
    iters += (uint32_t)it;
    fails += ok ? 0u : 1u;
}

template <class Model, class R, int KORD, bool LTE, bool SD = false>
__device__ inline void integrate(const Model& md, R x[Model::D], R gam[Model::D], double h_d,
                                 int M, R rtol, const R* __restrict__ floor_, int kmax,
                                 uint32_t& iters, uint32_t& fails)
{
    constexpr int D = Model::D;
    const R h = (R)h_d;
    R fl[D];                 // scale floors of the stopping test, in registers
#pragma unroll
    for (int i = 0; i < D; ++i) fl[i] = floor_[i];
    R h1[D], h2[D], h3[D];   // x_{m-2}, x_{m-3}, x_{m-4}
    if constexpr (LTE) {
#pragma unroll
        for (int i = 0; i < D; ++i) gam[i] = R(0);
    }
    int avail = 0;           // history beyond x_{m-1}
    // One step of the order-q formula.  QC > 0: q = QC = KORD is known at
    // compile time (every step after the ramp: coefficients and predictor are
    // constants); QC = 0: q from the history available (the ramp, and the
    // SDIRK start-up when SD).
    auto step = [&](auto qc) {
        constexpr int QC = decltype(qc)::value;
        const int q = QC > 0 ? QC : (avail < 1 ? 1 : (avail < KORD ? avail : KORD));
        const bool first = QC > 0 ? false : avail == 0;   // m = 1: Euler comparison value
        const BdfCoef co = bdf_coef(q);
        const R c = h * (R)co.beta;
        R psi[D], xp[D], xn[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            // the steady BDF2 and BDF3 steps with their fused multiply-adds
            // written out, so that unrolled copies round exactly as one step
            // does
            if constexpr (QC == 2) {
                psi[i] = rfma(x[i], -(R)co.a1, -((R)co.a2 * h1[i]));
                const R p = h2[i] + rfma(x[i], R(3), -(R(3) * h1[i]));
                xp[i] = p;
                xn[i] = p;
                continue;
            }
            if constexpr (QC == 3) {
                psi[i] = rfma(h2[i], -(R)co.a3, rfma(x[i], -(R)co.a1, -((R)co.a2 * h1[i])));
                const R p = rfma(h2[i], R(4), rfma(x[i], R(4), -(R(6) * h1[i]))) - h3[i];
                xp[i] = p;
                xn[i] = p;
                continue;
            }
            R s = -(R)co.a1 * x[i];
            if (KORD >= 2 && q >= 2) s -= (R)co.a2 * h1[i];
            if (KORD >= 3 && q >= 3) s -= (R)co.a3 * h2[i];
            psi[i] = s;
            R p = x[i];
            if (!first) {
                if (q == 1) p = R(2) * x[i] - h1[i];
                else if (KORD >= 2 && q == 2) p = R(3) * x[i] - R(3) * h1[i] + h2[i];
                else if (KORD >= 3) p = R(4) * x[i] - R(6) * h1[i] + R(4) * h2[i] - h3[i];
            }
            xp[i] = p;
            xn[i] = p;
        }
        typename Model::LU lu;
        if constexpr (SD && KORD >= 2 && QC == 0) {
            if (avail < KORD - 1) {
                // start-up step: the SDIRK stages, x_m the last one
                const Sdirk tb = sdirk_table<KORD>();
                R y[D], F[KORD][D], ps[D];
#pragma unroll
                for (int i = 0; i < D; ++i) y[i] = x[i];
#pragma unroll
                for (int sg = 0; sg < KORD; ++sg) {
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        R acc = R(0);
#pragma unroll
                        for (int j = 0; j < sg; ++j) acc += (R)tb.a[sg][j] * F[j][i];
                        ps[i] = x[i] + h * acc;
                    }
                    newton(md, y, ps, h * (R)tb.a[sg][sg], rtol, fl, kmax, lu, iters, fails);
                    md.rhs(y, F[sg]);
                }
                if constexpr (LTE) {
                    // the ramp's estimator: comparison value as above (Euler
                    // at m = 1), the ramp order's matrix at x_m
                    if (first) {
                        R f0[D];
                        md.rhs(x, f0);
#pragma unroll
                        for (int i = 0; i < D; ++i) xp[i] = x[i] + h * f0[i];
                    }
                    R fm[D];
                    md.eval(y, c, fm, lu);
                    const R kap = first ? R(0.5) : (R)co.kappa;
                    R e[D];
#pragma unroll
                    for (int i = 0; i < D; ++i) e[i] = y[i] - xp[i];
                    md.solve(lu, e);
                    if (first) md.solve(lu, e);
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        const R v = kap * e[i];
                        gam[i] += v * v;
                    }
                }
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    if (KORD >= 3) h3[i] = h2[i];
                    if (KORD >= 2) h2[i] = h1[i];
                    h1[i] = x[i];
                    x[i] = y[i];
                }
                avail = avail < KORD ? avail + 1 : KORD;
                return;
            }
        }
        // one exit (converged or kmax reached), so the loop is a plain
        // while-any-lane-active loop; the counts come from its exit state
        bool ok = false;
        int it = 0;
        do {
            R f[D];
            md.eval(xn, c, f, lu);
            if (LTE && first && it == 0) {
#pragma unroll
                for (int i = 0; i < D; ++i) xp[i] = x[i] + h * f[i];
            }
            R b[D];
#pragma unroll
            for (int i = 0; i < D; ++i) b[i] = (psi[i] + c * f[i]) - xn[i];
            md.solve(lu, b);
            ok = true;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                xn[i] += b[i];
                ok &= rabs(b[i]) <= rtol * rmax(rabs(xn[i]), fl[i]);
            }
            ++it;
        } while (!ok && it < kmax);
        iters += (uint32_t)it;
        fails += ok ? 0u : 1u;
        if constexpr (LTE) {
            const R kap = first ? R(0.5) : (R)co.kappa;
            R e[D];
#pragma unroll
            for (int i = 0; i < D; ++i) e[i] = xn[i] - xp[i];
            md.solve(lu, e);
            if (first) md.solve(lu, e);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const R v = kap * e[i];
                gam[i] += v * v;
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            if (KORD >= 3) h3[i] = h2[i];
            if (KORD >= 2) h2[i] = h1[i];
            h1[i] = x[i];
            x[i] = xn[i];
        }
        avail = avail < KORD ? avail + 1 : KORD;
    };
    int m = 1;
    for (; m <= M && avail < KORD; ++m) step(std::integral_constant<int, 0>{});
    if constexpr (sizeof(R) == 4 || D <= 4) {
        // unrolled by the history's rotation period (x_m and KORD older
        // states): the copies rename the history registers instead of moving
        // them (not for the large models in FP64, whose copies would spill).
        // The BDF1 step needs no written-out form: its products (x by 1 and
        // by 2) are exact, so any fusion rounds the same.
#pragma unroll(KORD + 1)
        for (; m <= M; ++m) step(std::integral_constant<int, KORD>{});
    } else {
        for (; m <= M; ++m) step(std::integral_constant<int, KORD>{});
    }
}

// ---------------------------------------------------------------------------
// Psi with the Adams-Moulton family: M fixed steps of the q-step formula
//   x_m = x_{m-1} + h (b0 f_m + b1 f_{m-1} + ... + bq f_{m-q}),
// q = min(KORD, m) (the derivatives f_0 .. f_{m-1} of the restarted
// interval), AM1 the trapezoidal rule.  The same Newton iteration as BDF on
// x = psi + h b0 f(x), started from x_{m-1} at m = 1 and from the degree-r
// extrapolation afterwards, r = min(q + 1, m - 1, 3).  f_m is evaluated once
// at the accepted x_m.  With LTE, gam accumulates the squared filtered Milne
// estimates kappa (I - h b0 J)^{-1} (x_m - x^(0)), x^(0) the extrapolation
// (error constant 1) or at m = 1 the Euler value (1/2, solved twice as for
// BDF), kappa = |C| / (C* + |C|) with |C| the formula's error constant.
// ---------------------------------------------------------------------------
struct AmCoef {
    double b0, b1, b2, b3;
    double errc;   // |C_{q+2}|
};

__device__ inline AmCoef am_coef(int q)
{
    if (q == 1) return {1.0 / 2.0, 1.0 / 2.0, 0.0, 0.0, 1.0 / 12.0};
    if (q == 2) return {5.0 / 12.0, 8.0 / 12.0, -1.0 / 12.0, 0.0, 1.0 / 24.0};
    return {9.0 / 24.0, 19.0 / 24.0, -5.0 / 24.0, 1.0 / 24.0, 19.0 / 720.0};
}

template <class Model, class R, int KORD, bool LTE>
__device__ inline void integrate_am(const Model& md, R x[Model::D], R gam[Model::D], double h_d, int M, R rtol,
                                    const R* __restrict__ floor_, int kmax, uint32_t& iters, uint32_t& fails)
{
    constexpr int D = Model::D;
    const R h = (R)h_d;
    R fl[D];
#pragma unroll
    for (int i = 0; i < D; ++i) fl[i] = floor_[i];
    R h1[D], h2[D], h3[D];       // x_{m-2}, x_{m-3}, x_{m-4}
    R f0[D], f1[D], f2[D];       // f_{m-1}, f_{m-2}, f_{m-3}
    if constexpr (LTE) {
#pragma unroll
        for (int i = 0; i < D; ++i) gam[i] = R(0);
    }
    md.rhs(x, f0);
    int avail = 0;               // x history beyond x_{m-1}
    // the steady steps (q = KORD, extrapolation degree RS) run with both known
    // at compile time; the first steps of the interval take them from m
    constexpr int RS = KORD + 1 < 3 ? KORD + 1 : 3;
    int m = 1;
    auto step = [&](auto steady) {
        constexpr bool ST = decltype(steady)::value;
        int q = KORD, r = RS;
        if constexpr (!ST) {
            q = m < KORD ? m : KORD;
            const int r0 = q + 1 < avail ? q + 1 : avail;
            r = r0 < 3 ? r0 : 3;
        }
        const AmCoef co = am_coef(q);
        const R c = h * (R)co.b0;
        R psi[D], xp[D], xn[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            if constexpr (ST && KORD == 1) {
                // the steady trapezoidal step with its fused multiply-adds
                // written out, so that unrolled copies round exactly as one
                // step does
                psi[i] = rfma((R)co.b1 * f0[i], h, x[i]);
                const R p = h2[i] + rfma(x[i], R(3), -(R(3) * h1[i]));
                xp[i] = p;
                xn[i] = p;
                continue;
            }
            R s = (R)co.b1 * f0[i];
            if (KORD >= 2 && q >= 2) s += (R)co.b2 * f1[i];
            if (KORD >= 3 && q >= 3) s += (R)co.b3 * f2[i];
            psi[i] = x[i] + h * s;
            R p;
            if (r == 0) p = x[i] + h * f0[i];
            else if (r == 1) p = R(2) * x[i] - h1[i];
            else if (r == 2) p = R(3) * x[i] - R(3) * h1[i] + h2[i];
            else p = R(4) * x[i] - R(6) * h1[i] + R(4) * h2[i] - h3[i];
            xp[i] = p;
            xn[i] = r == 0 ? x[i] : p;
        }
        typename Model::LU lu;
        bool ok = false;
        int it = 0;
        do {
            R f[D];
            md.eval(xn, c, f, lu);
            R b[D];
#pragma unroll
            for (int i = 0; i < D; ++i) b[i] = (psi[i] + c * f[i]) - xn[i];
            md.solve(lu, b);
            ok = true;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                xn[i] += b[i];
                ok &= rabs(b[i]) <= rtol * rmax(rabs(xn[i]), fl[i]);
            }
            ++it;
        } while (!ok && it < kmax);
        iters += (uint32_t)it;
        fails += ok ? 0u : 1u;
        if constexpr (LTE) {
            const R cstar = r == 0 ? R(0.5) : R(1);
            const R kap = (R)co.errc / (cstar + (R)co.errc);
            R e[D];
#pragma unroll
            for (int i = 0; i < D; ++i) e[i] = xn[i] - xp[i];
            md.solve(lu, e);
            if (r == 0) md.solve(lu, e);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const R v = kap * e[i];
                gam[i] += v * v;
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            h3[i] = h2[i];
            h2[i] = h1[i];
            h1[i] = x[i];
            x[i] = xn[i];
            if (KORD >= 3) f2[i] = f1[i];
            if (KORD >= 2) f1[i] = f0[i];
        }
        md.rhs(x, f0);
        avail = avail < 3 ? avail + 1 : 3;
    };
    for (; m <= M && !(m >= KORD && avail >= RS); ++m) step(std::false_type{});
    // AM1 unrolled by its history's rotation period (x_m, x_{m-1}, x_{m-2}):
    // the copies rename the history registers instead of moving them
    if constexpr (KORD == 1 && (sizeof(R) == 4 || D <= 4)) {
#pragma unroll(3)
        for (; m <= M; ++m) step(std::true_type{});
    } else {
        for (; m <= M; ++m) step(std::true_type{});
    }
}

// Psi of either LMM family (LMM 0 BDF, 1 Adams-Moulton, 2 BDF with the SDIRK start-up)
template <class Model, class R, int KORD, bool LTE, int LMM>
__device__ inline void integrate_lmm(const Model& md, R x[Model::D], R gam[Model::D], double h_d, int M, R rtol,
                                     const R* __restrict__ floor_, int kmax, uint32_t& iters, uint32_t& fails)
{
    if constexpr (LMM == 1) integrate_am<Model, R, KORD, LTE>(md, x, gam, h_d, M, rtol, floor_, kmax, iters, fails);
    else if constexpr (LMM == 2) integrate<Model, R, KORD, LTE, true>(md, x, gam, h_d, M, rtol, floor_, kmax, iters, fails);
    else integrate<Model, R, KORD, LTE>(md, x, gam, h_d, M, rtol, floor_, kmax, iters, fails);
}

// Gaussian log-likelihood of the observed components, constants dropped;
// -inf for a non-finite observed state.  Loops are unrolled over the largest
// sizes (MOBS_KIN observed components) so every index into the lane's
// registers is static.
template <class R, int D>
__device__ inline double loglik(const R (&x)[D], const int32_t* obs, const double (&y)[MMAX],
                                const double (&sg)[MMAX], int m)
{
    double s = 0.0;
    bool finite = true;
#pragma unroll
    for (int i = 0; i < MOBS_KIN; ++i) {
        if (i < m) {
            const int k = obs[i];
            R xv = x[0];
#pragma unroll
            for (int c = 1; c < D; ++c)
                if (c == k) xv = x[c];
            const double v = (double)xv;
            finite = finite && isfinite(v);
            const double r = (y[i] - v) / sg[i];
            s += r * r;
        }
    }
    return finite ? -0.5 * s : -INFINITY;
}

}  // namespace pf

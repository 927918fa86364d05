/*
 * pf_oracle.c -- plain, slow FP64 reference of the LMM PF-SMC sampler
 * (Arnold, Calvetti & Somersalo, "Vectorized and Parallel Particle Filter SMC
 * Parameter Estimation for Stiff ODEs", Sec. 2, Algorithm 1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source with the HIP library
 * (no headers, tables or helpers): every formula below is written out again
 * from the paper and from the published definitions it cites.
 *
 * Everything is double precision.  Particles are stored array-of-structures
 * (x[n*d + i], theta[n*p + i]) because that is the plainest layout; loops over
 * particles carry an OpenMP pragma and nothing else.
 *
 * Models: Robertson kinetics and the compartment chain (stiffness that
 * depends on the parameters), and the 2D periodic advection-diffusion system
 * of Sec. 4 (uniform stiffness, up to 39 x 39 grid values per particle).
 *
 * Readings of points the paper leaves open are marked "Reading:" where they
 * are used.  Parity status of each function is in its comment; the one piece
 * with no pin beyond internal consistency is the innovation-variance reading
 * (the paper defers its formula to a companion paper): parity unpinned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* largest sizes: states (the 39 x 39 advection-diffusion grid), parameters,
 * observed components.  Vectors of these sizes live on the stack; d x d
 * matrices are allocated per call. */
#define OR_DMAX 1521
#define OR_PMAX 12
#define OR_MMAX 32

/* status codes (plain ints; mirrored by the Python wrapper) */
#define OR_OK 0
#define OR_EINVAL 1
#define OR_EDEGENERATE 4

/* ------------------------------------------------------------------------- */
/* Counter-based RNG: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel    */
/* random numbers: as easy as 1, 2, 3", SC'11).  A round maps the counter     */
/* (c0,c1,c2,c3) with key (k0,k1) to                                          */
/*   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));          */
/* the key is bumped by the Weyl constants between rounds; ten rounds.        */
/* ------------------------------------------------------------------------- */
static const uint64_t PHX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHX_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PHX_W1 = 0xBB67AE8584CAA73BULL;

void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PHX_W0; k1 += PHX_W1; }
        unsigned __int128 p0 = (unsigned __int128)PHX_M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)PHX_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform on the open interval (0,1) from the top 53 bits */
double or_u01(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1p-53; }

/*
 * Gaussian draws of one purpose: counter (step, particle, purpose, block),
 * key (seed, 0).  A block gives four words -> four uniforms u0..u3 -> two
 * Box-Muller pairs (Box & Muller 1958):
 *   z0 = sqrt(-2 ln u0) cos(2 pi u1),  z1 = sqrt(-2 ln u0) sin(2 pi u1),
 *   z2 = sqrt(-2 ln u2) cos(2 pi u3),  z3 = sqrt(-2 ln u2) sin(2 pi u3).
 * Normal number k of the purpose comes from block k/4, slot k%4.
 */
void or_normals(uint64_t seed, uint64_t step, uint64_t particle, uint64_t purpose,
                int count, double* out)
{
    const double two_pi = 6.283185307179586476925286766559;
    uint64_t key[2] = {seed, 0};
    for (int b = 0; 4 * b < count; ++b) {
        uint64_t ctr[4] = {step, particle, purpose, (uint64_t)b};
        uint64_t w[4];
        or_philox4x64(ctr, key, w);
        double u0 = or_u01(w[0]), u1 = or_u01(w[1]), u2 = or_u01(w[2]), u3 = or_u01(w[3]);
        double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
        double z[4] = {r0 * cos(two_pi * u1), r0 * sin(two_pi * u1),
                       r1 * cos(two_pi * u3), r1 * sin(two_pi * u3)};
        for (int s = 0; s < 4 && 4 * b + s < count; ++s) out[4 * b + s] = z[s];
    }
}

/* RNG purposes (third counter word) */
enum { PUR_PRIOR = 1, PUR_RESAMPLE = 2, PUR_PROLIF = 3, PUR_INNOV = 4 };

/* ------------------------------------------------------------------------- */
/* Backward differentiation formulas (Sec. 2.1: implicit LMMs for the stiff   */
/* propagation).  Normalised with the coefficient of x_m equal to one:        */
/*   x_m + sum_{i=1..q} alpha_i x_{m-i} = h beta f(x_m),                       */
/* error constant C_{q+1}: the residual of the formula on the exact solution  */
/* is C_{q+1} h^{q+1} x^{(q+1)} + O(h^{q+2}).  Textbook values.               */
/* ------------------------------------------------------------------------- */
int or_bdf(int q, double alpha[4], double* beta, double* errc)
{
    for (int i = 0; i < 4; ++i) alpha[i] = 0.0;
    alpha[0] = 1.0;
    switch (q) {
    case 1: alpha[1] = -1.0; *beta = 1.0; *errc = -1.0 / 2.0; return 0;
    case 2: alpha[1] = -4.0 / 3.0; alpha[2] = 1.0 / 3.0; *beta = 2.0 / 3.0; *errc = -2.0 / 9.0; return 0;
    case 3: alpha[1] = -18.0 / 11.0; alpha[2] = 9.0 / 11.0; alpha[3] = -2.0 / 11.0;
            *beta = 6.0 / 11.0; *errc = -3.0 / 22.0; return 0;
    default: return OR_EINVAL;
    }
}

/* Adams-Moulton, q steps (order q + 1):                                     */
/*   x_m = x_{m-1} + h (beta_0 f_m + beta_1 f_{m-1} + ... + beta_q f_{m-q}),  */
/* AM1 the trapezoidal rule; errc = |C_{q+2}|, the local error constant.      */
int or_am(int q, double beta[4], double* errc)
{
    for (int i = 0; i < 4; ++i) beta[i] = 0.0;
    switch (q) {
    case 1: beta[0] = 1.0 / 2.0; beta[1] = 1.0 / 2.0; *errc = 1.0 / 12.0; return 0;
    case 2: beta[0] = 5.0 / 12.0; beta[1] = 8.0 / 12.0; beta[2] = -1.0 / 12.0; *errc = 1.0 / 24.0; return 0;
    case 3: beta[0] = 9.0 / 24.0; beta[1] = 19.0 / 24.0; beta[2] = -5.0 / 24.0; beta[3] = 1.0 / 24.0;
            *errc = 19.0 / 720.0; return 0;
    default: return OR_EINVAL;
    }
}

/* weights of the degree-q polynomial through x_{m-1},...,x_{m-1-q} evaluated
 * one step ahead: (-1)^i binom(q+1, i+1) for x_{m-1-i}. */
static void or_extrap_weights(int q, double w[4])
{
    static const double tab[4][4] = {{1, 0, 0, 0}, {2, -1, 0, 0}, {3, -3, 1, 0}, {4, -6, 4, -1}};
    for (int i = 0; i < 4; ++i) w[i] = tab[q][i];
}

/* ------------------------------------------------------------------------- */
/* Models: right-hand side f(x; k) and Jacobian J = df/dx (row-major d x d).  */
/* `k` is the full vector of rate constants; `mc` the fixed model constants. */
/* ------------------------------------------------------------------------- */
enum { MODEL_DECAY = 0, MODEL_ROBERTSON = 1, MODEL_CHAIN = 2, MODEL_ADVDIFF = 3 };

/* x_i' = -k_i x_i (test problem with a closed form; d = p) */
static void rhs_decay(int d, const double* x, const double* k, double* f, double* J)
{
    for (int i = 0; i < d; ++i) f[i] = -k[i] * x[i];
    if (J) {
        for (int i = 0; i < d * d; ++i) J[i] = 0.0;
        for (int i = 0; i < d; ++i) J[i * d + i] = -k[i];
    }
}

/* Robertson kinetics: A -> B (k1), 2B -> B + C (k2), B + C -> A + C (k3) */
static void rhs_robertson(const double* x, const double* k, double* f, double* J)
{
    double k1 = k[0], k2 = k[1], k3 = k[2];
    f[0] = -k1 * x[0] + k3 * x[1] * x[2];
    f[1] = k1 * x[0] - k2 * x[1] * x[1] - k3 * x[1] * x[2];
    f[2] = k2 * x[1] * x[1];
    if (J) {
        J[0] = -k1; J[1] = k3 * x[2];                    J[2] = k3 * x[1];
        J[3] = k1;  J[4] = -2.0 * k2 * x[1] - k3 * x[2]; J[5] = -k3 * x[1];
        J[6] = 0.0; J[7] = 2.0 * k2 * x[1];              J[8] = 0.0;
    }
}

/* Compartment chain with Michaelis-Menten losses:
 *   x_i' = k_{i-1} x_{i-1} - k_i x_i - V_i x_i / (K_i + x_i),
 * with a constant unit influx into the first compartment.
 * mc layout: [V_1..V_d, K_1..K_d]. */
static void rhs_chain(int d, const double* x, const double* k, const double* mc,
                      double* f, double* J)
{
    const double* V = mc;
    const double* K = mc + d;
    for (int i = 0; i < d; ++i) {
        double in = (i == 0) ? 1.0 : k[i - 1] * x[i - 1];
        f[i] = in - k[i] * x[i] - V[i] * x[i] / (K[i] + x[i]);
    }
    if (J) {
        for (int i = 0; i < d * d; ++i) J[i] = 0.0;
        for (int i = 0; i < d; ++i) {
            double den = K[i] + x[i];
            J[i * d + i] = -k[i] - V[i] * K[i] / (den * den);
            if (i > 0) J[i * d + i - 1] = k[i - 1];
        }
    }
}

/* 2D periodic advection-diffusion (Sec. 4), semi-discretised as dU/dt = L U:
 *   L = -(k1^2 B1^T B1 + k1 k3 (B1^T B2 + B2^T B1) + (k2^2 + k3^2) B2^T B2)
 *       + c1 B1 + c2 B2,
 * B1 = I (x) l, B2 = l (x) I, with l the nt x nt periodic difference matrix
 * of Sec. 4 (1 on the diagonal, -1 below it and in the top-right corner):
 * (l v)_i = v_i - v_{i-1 mod nt}, (l^T v)_i = v_i - v_{i+1 mod nt}.
 * Reading (stacking): U[iy * nt + ix], x fastest, so that the Kronecker
 * factor I (x) l acts along x as B1 stands for d/dx.  Reading (scale): l as
 * printed, without a 1/dx factor (coefficients in grid units).
 * theta = (k1, k2, k3, c1, c2) is used as is (the paper estimates these
 * parameters, not their logarithms); mc[0] = nt, d = nt^2.
 * f = L x through the factors; J = L, assembled column by column as L e_j. */
static void diff_x(int nt, const double* v, double* o, int transposed)
{
    for (int iy = 0; iy < nt; ++iy)
        for (int ix = 0; ix < nt; ++ix) {
            int nb = transposed ? (ix + 1) % nt : (ix + nt - 1) % nt;
            o[iy * nt + ix] = v[iy * nt + ix] - v[iy * nt + nb];
        }
}

static void diff_y(int nt, const double* v, double* o, int transposed)
{
    for (int iy = 0; iy < nt; ++iy) {
        int nb = transposed ? (iy + 1) % nt : (iy + nt - 1) % nt;
        for (int ix = 0; ix < nt; ++ix) o[iy * nt + ix] = v[iy * nt + ix] - v[nb * nt + ix];
    }
}

static void advdiff_apply(int nt, const double* th, const double* v, double* o)
{
    int d = nt * nt;
    double b1[OR_DMAX], b2[OR_DMAX], t11[OR_DMAX], t12[OR_DMAX], t21[OR_DMAX], t22[OR_DMAX];
    double k1 = th[0], k2 = th[1], k3 = th[2], c1 = th[3], c2 = th[4];
    diff_x(nt, v, b1, 0);       /* B1 v */
    diff_y(nt, v, b2, 0);       /* B2 v */
    diff_x(nt, b1, t11, 1);     /* B1^T B1 v */
    diff_x(nt, b2, t12, 1);     /* B1^T B2 v */
    diff_y(nt, b1, t21, 1);     /* B2^T B1 v */
    diff_y(nt, b2, t22, 1);     /* B2^T B2 v */
    for (int i = 0; i < d; ++i)
        o[i] = -(k1 * k1 * t11[i] + k1 * k3 * (t12[i] + t21[i]) + (k2 * k2 + k3 * k3) * t22[i])
               + c1 * b1[i] + c2 * b2[i];
}

static void rhs_advdiff(int d, const double* x, const double* theta, const double* mc, double* f, double* J)
{
    int nt = (int)mc[0];
    advdiff_apply(nt, theta, x, f);
    if (J) {
        double e[OR_DMAX], col[OR_DMAX];
        for (int i = 0; i < d; ++i) e[i] = 0.0;
        for (int j = 0; j < d; ++j) {
            e[j] = 1.0;
            advdiff_apply(nt, theta, e, col);
            e[j] = 0.0;
            for (int i = 0; i < d; ++i) J[i * d + j] = col[i];
        }
    }
}

/*
 * Model description.  Rate constants of the kinetic models: the first p are
 * exp(theta); the rest (chain only) are fixed and come from `rates_fixed`.
 */
typedef struct {
    int model;          /* MODEL_* */
    int d;              /* state dimension */
    int p;              /* number of estimated log-parameters */
    const double* mc;   /* chain: [V(d), K(d)]; unused otherwise */
    const double* rates_fixed; /* chain: full k(d); entries p..d-1 are used */
} or_model;

void or_rhs(int model, int d, int p, const double* mc, const double* rates_fixed,
            const double* x, const double* theta, double* f, double* J)
{
    if (model == MODEL_ADVDIFF) {
        rhs_advdiff(d, x, theta, mc, f, J);
        return;
    }
    double k[OR_DMAX];
    int nk = (model == MODEL_ROBERTSON) ? 3 : d;
    for (int i = 0; i < nk; ++i) k[i] = (i < p) ? exp(theta[i]) : rates_fixed[i];
    if (model == MODEL_DECAY) rhs_decay(d, x, k, f, J);
    else if (model == MODEL_ROBERTSON) rhs_robertson(x, k, f, J);
    else rhs_chain(d, x, k, mc, f, J);
}

/* ------------------------------------------------------------------------- */
/* Dense LU with partial pivoting: solve A z = b (A row-major, destroyed).    */
/* Returns 0, or -1 if a pivot is exactly zero or not finite.                 */
/* ------------------------------------------------------------------------- */
int or_lu_solve(int d, double* A, double* b)
{
    for (int c = 0; c < d; ++c) {
        int piv = c;
        double best = fabs(A[c * d + c]);
        for (int r = c + 1; r < d; ++r)
            if (fabs(A[r * d + c]) > best) { best = fabs(A[r * d + c]); piv = r; }
        if (!(best > 0.0) || !isfinite(best)) return -1;
        if (piv != c) {
            for (int j = 0; j < d; ++j) { double t = A[c * d + j]; A[c * d + j] = A[piv * d + j]; A[piv * d + j] = t; }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < d; ++r) {
            double l = A[r * d + c] / A[c * d + c];
            A[r * d + c] = 0.0;
            for (int j = c + 1; j < d; ++j) A[r * d + j] -= l * A[c * d + j];
            b[r] -= l * b[c];
        }
    }
    for (int r = d - 1; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < d; ++j) s -= A[r * d + j] * b[j];
        b[r] = s / A[r * d + r];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Psi: propagate one particle over one observation interval with M fixed    */
/* BDF steps of size h (Algorithm 1, steps 2 and 4(d)); optionally also the   */
/* LMM local-error estimate that sets the innovation variance (step 4(b)).    */
/*                                                                            */
/* Reading (start-up): Psi only receives x_j, so every interval restarts from */
/* a single value.  Step m (1-based) uses order q = max(1, min(k, m-1)): the  */
/* order a degree-q extrapolation predictor through the available history     */
/* can support.  Step 1 uses the explicit Euler predictor x_0 + h f(x_0).     */
/*                                                                            */
/* Reading (Newton): full Newton on G(x) = x - psi - h beta f(x) from the     */
/* predictor, analytic Jacobian refreshed every iteration, solve              */
/* (I - h beta J) dx = -G, x += dx; stop after the first iteration with       */
/* max_i |dx_i| / max(|x_i|, floor_i) <= rtol, or after kmax iterations.      */
/*                                                                            */
/* Reading (Newton start): the predictor below at steps m >= 2; at step 1     */
/* the previous value x_0 itself (an explicit Euler guess is unstable for the */
/* stiff components when h |lambda| >> 1).                                    */
/*                                                                            */
/* Reading (innovation variance, parity unpinned against the paper): the     */
/* Milne-device estimate of each step's local error, filtered through the     */
/* Newton matrix so that stiff components are not over-estimated:             */
/*   e_m = |C_{q+1}| / (C* + |C_{q+1}|) * (I - h beta J)^{-1} (x_m - x_m^(0)), */
/* with x^(0) the degree-q extrapolation (error constant C* = 1) or, at step  */
/* 1, the Euler value x_0 + h f(x_0) (C* = 1/2); J is the Jacobian of the     */
/* last Newton iteration.  At step 1 the filter is applied twice: the Euler   */
/* value's own error in a stiff mode is (1 - h lambda) times larger than a    */
/* stable predictor's, so a single filter leaves an estimate of half the      */
/* mode's amplitude, while two bring it to the order of the true local error  */
/* (1 / |h lambda| of the amplitude) and still tend to Milne's estimate as    */
/* h -> 0.  Steps add as independent variances:                               */
/*   Gamma = diag(sum_m e_m^2).                                               */
/*                                                                            */
/* `hist` (optional, pins only): q_hist earlier values x_{-1},...,x_{-q_hist} */
/* on the same grid, so that the formula runs at full order from step 1.      */
/* ------------------------------------------------------------------------- */
typedef struct {
    long newton_iters;  /* total Newton iterations */
    long newton_fails;  /* steps that hit kmax without meeting the test */
    long lu_fails;      /* singular or non-finite pivots */
} or_psi_stats;

/* ------------------------------------------------------------------------- */
/* Order-preserving start-up (reading R2-S): the steps of an interval that    */
/* lack the history for the full BDF order, m = 1 .. k-1, are taken with an   */
/* L-stable, stiffly accurate SDIRK method of order k (Alexander 1977): for   */
/* k = 2 two stages with gamma = 1 - 1/sqrt(2); for k = 3 three stages with   */
/* gamma the root of gamma^3 - 3 gamma^2 + 3 gamma / 2 - 1/6 in (1/6, 1/2).   */
/* Stage i solves Y = x_{m-1} + h sum_{j<i} a_ij f(Y_j) + h gamma f(Y) by the */
/* same Newton iteration (started from x_{m-1}, then from the previous        */
/* stage); x_m is the last stage.  The innovation variance of these steps     */
/* keeps the ramp's estimator (the comparison value and kappa of the BDF     */
/* order the ramp would use), with J at x_m.                                  */
/* ------------------------------------------------------------------------- */
int or_sdirk(int k, double A[3][3], int* stages)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = 0.0;
    if (k == 2) {
        const double g = 1.0 - sqrt(0.5);
        A[0][0] = g;
        A[1][0] = 1.0 - g; A[1][1] = g;
        *stages = 2;
        return 0;
    }
    if (k == 3) {
        /* the root in (1/6, 1/2), by bisection on the cubic */
        double lo = 1.0 / 6.0, hi = 0.5;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            double v = ((mid - 3.0) * mid + 1.5) * mid - 1.0 / 6.0;
            double vlo = ((lo - 3.0) * lo + 1.5) * lo - 1.0 / 6.0;
            if ((v > 0) == (vlo > 0)) lo = mid;
            else hi = mid;
        }
        const double g = 0.5 * (lo + hi);
        A[0][0] = g;
        A[1][0] = (1.0 - g) / 2.0; A[1][1] = g;
        A[2][0] = -(6.0 * g * g - 16.0 * g + 1.0) / 4.0;
        A[2][1] = (6.0 * g * g - 20.0 * g + 5.0) / 4.0;
        A[2][2] = g;
        *stages = 3;
        return 0;
    }
    return OR_EINVAL;
}

/* one Newton solve of Y = psi + c f(Y) from the guess in x (overwritten); the
 * matrix of the last iteration is left in Alast */
static int newton_solve(int model, int d, int p, const double* mc, const double* rates_fixed,
                        const double* theta, const double* psi, double c, double rtol, int kmax,
                        const double* floor_, double* x, double* Alast, double* J, double* A,
                        or_psi_stats* st)
{
    int conv = 0;
    for (int it = 0; it < kmax; ++it) {
        double f[OR_DMAX], rhs[OR_DMAX];
        or_rhs(model, d, p, mc, rates_fixed, x, theta, f, J);
        for (int i = 0; i < d; ++i) rhs[i] = -(x[i] - psi[i] - c * f[i]);
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) A[a * d + b] = (a == b ? 1.0 : 0.0) - c * J[a * d + b];
        if (Alast) memcpy(Alast, A, sizeof(double) * d * d);
        if (st) st->newton_iters++;
        if (or_lu_solve(d, A, rhs) != 0) {
            if (st) st->lu_fails++;
            for (int i = 0; i < d; ++i) x[i] = NAN;
            return 0;
        }
        double worst = 0.0;
        for (int i = 0; i < d; ++i) {
            x[i] += rhs[i];
            double sc = fabs(x[i]) > floor_[i] ? fabs(x[i]) : floor_[i];
            double r = fabs(rhs[i]) / sc;
            if (r != r) r = INFINITY;
            if (r > worst) worst = r;
        }
        if (worst <= rtol) { conv = 1; break; }
    }
    if (!conv && st) st->newton_fails++;
    return conv;
}

static int or_psi_bdf(int model, int d, int p, const double* mc, const double* rates_fixed,
                      const double* x0, const double* theta, double h, int M, int k,
                      int want_lte, double rtol, int kmax, const double* floor_,
                      const double* hist, int q_hist, int sdirk_start,
                      double* x_out, double* gamma_out, or_psi_stats* st);

int or_psi(int model, int d, int p, const double* mc, const double* rates_fixed,
           const double* x0, const double* theta, double h, int M, int k,
           int want_lte, double rtol, int kmax, const double* floor_,
           const double* hist, int q_hist,
           double* x_out, double* gamma_out, or_psi_stats* st)
{
    if (d < 1 || d > OR_DMAX) return OR_EINVAL;
    return or_psi_bdf(model, d, p, mc, rates_fixed, x0, theta, h, M, k, want_lte, rtol, kmax, floor_, hist,
                      q_hist, 0, x_out, gamma_out, st);
}

static int or_psi_bdf(int model, int d, int p, const double* mc, const double* rates_fixed,
                      const double* x0, const double* theta, double h, int M, int k,
                      int want_lte, double rtol, int kmax, const double* floor_,
                      const double* hist, int q_hist, int sdirk_start,
                      double* x_out, double* gamma_out, or_psi_stats* st)
{
    /* H[0] = x_{m-1}, H[1] = x_{m-2}, ... (ring of up to 4 values) */
    double H[4][OR_DMAX];
    int nh = 1;
    memcpy(H[0], x0, sizeof(double) * d);
    if (hist) {
        for (int r = 0; r < q_hist && r < 3; ++r) memcpy(H[r + 1], hist + r * d, sizeof(double) * d);
        nh = 1 + (q_hist < 3 ? q_hist : 3);
    }
    double gam[OR_DMAX];
    for (int i = 0; i < d; ++i) gam[i] = 0.0;
    /* d x d work matrices: the last Newton matrix, J, A */
    double* Alast = (double*)malloc(sizeof(double) * 3 * (size_t)d * d);
    if (!Alast) return OR_EINVAL;
    double* J = Alast + (size_t)d * d;
    double* A = J + (size_t)d * d;

    for (int m = 1; m <= M; ++m) {
        int avail = nh - 1;               /* past values beyond x_{m-1} */
        int q = avail < k ? avail : k;
        if (q < 1) q = 1;
        double alpha[4], beta, errc;
        or_bdf(q, alpha, &beta, &errc);

        /* predictor x^(0) and its error constant */
        double xp[OR_DMAX], cstar;
        if (avail == 0) {
            double f0[OR_DMAX];
            or_rhs(model, d, p, mc, rates_fixed, H[0], theta, f0, NULL);
            for (int i = 0; i < d; ++i) xp[i] = H[0][i] + h * f0[i];
            cstar = 0.5;
        } else {
            double w[4];
            or_extrap_weights(q, w);
            for (int i = 0; i < d; ++i) {
                double s = 0.0;
                for (int r = 0; r <= q; ++r) s += w[r] * H[r][i];
                xp[i] = s;
            }
            cstar = 1.0;
        }

        /* psi = -sum_{i>=1} alpha_i x_{m-i} */
        double psi[OR_DMAX];
        for (int i = 0; i < d; ++i) {
            double s = 0.0;
            for (int r = 1; r <= q; ++r) s -= alpha[r] * H[r - 1][i];
            psi[i] = s;
        }

        double x[OR_DMAX];
        double c = h * beta;
        if (sdirk_start && k >= 2 && avail < k - 1) {
            /* start-up step by SDIRK of order k (x_m = last stage) */
            double Asd[3][3], F[3][OR_DMAX];
            int ns;
            or_sdirk(k, Asd, &ns);
            memcpy(x, H[0], sizeof(double) * d);
            for (int sg = 0; sg < ns; ++sg) {
                double ps[OR_DMAX];
                for (int i = 0; i < d; ++i) {
                    double sacc = 0.0;
                    for (int j = 0; j < sg; ++j) sacc += Asd[sg][j] * F[j][i];
                    ps[i] = H[0][i] + h * sacc;
                }
                newton_solve(model, d, p, mc, rates_fixed, theta, ps, h * Asd[sg][sg], rtol, kmax, floor_, x,
                             NULL, J, A, st);
                or_rhs(model, d, p, mc, rates_fixed, x, theta, F[sg], NULL);
            }
            if (want_lte) {
                /* the ramp's estimator, with the ramp order's matrix at x_m */
                double f[OR_DMAX];
                or_rhs(model, d, p, mc, rates_fixed, x, theta, f, J);
                for (int a = 0; a < d; ++a)
                    for (int b = 0; b < d; ++b) Alast[a * d + b] = (a == b ? 1.0 : 0.0) - c * J[a * d + b];
                double kap = fabs(errc) / (cstar + fabs(errc));
                double e[OR_DMAX];
                for (int i = 0; i < d; ++i) e[i] = x[i] - xp[i];
                if (avail == 0) memcpy(A, Alast, sizeof(double) * d * d);
                if (or_lu_solve(d, Alast, e) != 0 || (avail == 0 && or_lu_solve(d, A, e) != 0))
                    for (int i = 0; i < d; ++i) e[i] = NAN;
                for (int i = 0; i < d; ++i) {
                    double ei = kap * e[i];
                    gam[i] += ei * ei;
                }
            }
            for (int r = 3; r > 0; --r) memcpy(H[r], H[r - 1], sizeof(double) * d);
            memcpy(H[0], x, sizeof(double) * d);
            if (nh < 4) nh++;
            continue;
        }

        /* Newton, from x_0 at step 1 and from the predictor afterwards */
        memcpy(x, avail == 0 ? H[0] : xp, sizeof(double) * d);
        int conv = 0;
        for (int it = 0; it < kmax; ++it) {
            double f[OR_DMAX], rhs[OR_DMAX];
            or_rhs(model, d, p, mc, rates_fixed, x, theta, f, J);
            for (int i = 0; i < d; ++i) rhs[i] = -(x[i] - psi[i] - c * f[i]);
            for (int r = 0; r < d; ++r)
                for (int s = 0; s < d; ++s) A[r * d + s] = (r == s ? 1.0 : 0.0) - c * J[r * d + s];
            memcpy(Alast, A, sizeof(double) * d * d);
            if (st) st->newton_iters++;
            if (or_lu_solve(d, A, rhs) != 0) {
                if (st) st->lu_fails++;
                for (int i = 0; i < d; ++i) x[i] = NAN;
                break;
            }
            double worst = 0.0;
            for (int i = 0; i < d; ++i) {
                x[i] += rhs[i];
                double sc = fabs(x[i]) > floor_[i] ? fabs(x[i]) : floor_[i];
                double r = fabs(rhs[i]) / sc;
                if (r != r) r = INFINITY;       /* NaN counts as "not converged" */
                if (r > worst) worst = r;
            }
            if (worst <= rtol) { conv = 1; break; }
        }
        if (!conv && st) st->newton_fails++;

        if (want_lte) {
            double kap = fabs(errc) / (cstar + fabs(errc));
            double e[OR_DMAX];
            for (int i = 0; i < d; ++i) e[i] = x[i] - xp[i];
            /* step 1: the Euler comparison is filtered twice */
            if (avail == 0) memcpy(A, Alast, sizeof(double) * d * d);
            if (or_lu_solve(d, Alast, e) != 0 || (avail == 0 && or_lu_solve(d, A, e) != 0))
                for (int i = 0; i < d; ++i) e[i] = NAN;
            for (int i = 0; i < d; ++i) {
                double ei = kap * e[i];
                gam[i] += ei * ei;
            }
        }

        /* shift history */
        for (int r = 3; r > 0; --r) memcpy(H[r], H[r - 1], sizeof(double) * d);
        memcpy(H[0], x, sizeof(double) * d);
        if (nh < 4) nh++;
    }
    free(Alast);
    memcpy(x_out, H[0], sizeof(double) * d);
    if (gamma_out) memcpy(gamma_out, gam, sizeof(double) * d);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Psi with the Adams-Moulton family (the paper's other implicit LMMs).      */
/*                                                                            */
/* Reading (naming): AMk is the k-step Adams-Moulton formula, of order k + 1 */
/* (AM1 = trapezoidal rule), so that AM1 differs from BDF1 = backward Euler   */
/* (the paper times them differently) and "the first three of each family"   */
/* count steps as for AB and BDF.                                             */
/* Reading (start-up): as for BDF, each interval restarts from x_j alone;     */
/* step m has the derivatives f_0 .. f_{m-1} and uses q = min(k, m) steps.    */
/* f_m = f(x_m) is evaluated once at the accepted x_m.                        */
/* Reading (Newton): the same full Newton as BDF on                           */
/* G(x) = x - psi - h beta_0 f(x), psi = x_{m-1} + h sum_{i>=1} beta_i f_{m-i}, */
/* started from x_0 at step 1 and from the extrapolation below afterwards.    */
/* Reading (innovation variance, parity unpinned against the paper): Milne's */
/* device with a polynomial predictor instead of an Adams-Bashforth one (an   */
/* explicit derivative-based predictor is unstable for the stiff components   */
/* when h |lambda| >> 1): x^(0) the degree-r extrapolation through            */
/* x_{m-1} .. x_{m-1-r}, r = min(q + 1, m - 1, 3) (error constant 1), or at   */
/* step 1 the Euler value x_0 + h f_0 (error constant 1/2), filtered twice   */
/* as for BDF;                                                                */
/*   e_m = |C| / (C* + |C|) (I - h beta_0 J)^{-1} (x_m - x^(0)),              */
/*   Gamma = diag(sum_m e_m^2).                                               */
/* `hist` (pins only): earlier values x_{-1}, ... on the same grid; their     */
/* derivatives join the history so the formula runs at full order.           */
/* ------------------------------------------------------------------------- */
int or_psi_am(int model, int d, int p, const double* mc, const double* rates_fixed,
              const double* x0, const double* theta, double h, int M, int k,
              int want_lte, double rtol, int kmax, const double* floor_,
              const double* hist, int q_hist,
              double* x_out, double* gamma_out, or_psi_stats* st)
{
    /* H[0] = x_{m-1}, H[1] = x_{m-2}, ...; F[r] = f(H[r]) */
    if (d < 1 || d > OR_DMAX) return OR_EINVAL;
    double H[5][OR_DMAX], F[4][OR_DMAX];
    int nh = 1;
    memcpy(H[0], x0, sizeof(double) * d);
    if (hist) {
        for (int r = 0; r < q_hist && r < 4; ++r) memcpy(H[r + 1], hist + r * d, sizeof(double) * d);
        nh = 1 + (q_hist < 4 ? q_hist : 4);
    }
    for (int r = 0; r < nh && r < 4; ++r) or_rhs(model, d, p, mc, rates_fixed, H[r], theta, F[r], NULL);
    double gam[OR_DMAX];
    for (int i = 0; i < d; ++i) gam[i] = 0.0;
    /* d x d work matrices: the last Newton matrix, J, A */
    double* Alast = (double*)malloc(sizeof(double) * 3 * (size_t)d * d);
    if (!Alast) return OR_EINVAL;
    double* J = Alast + (size_t)d * d;
    double* A = J + (size_t)d * d;

    for (int m = 1; m <= M; ++m) {
        int nf = nh < 4 ? nh : 4;             /* derivatives available: f_{m-1} .. */
        int q = nf < k ? nf : k;
        double beta[4], errc;
        or_am(q, beta, &errc);

        /* comparison value x^(0) and its error constant; Newton start */
        double xp[OR_DMAX], cstar;
        int r = nh - 1 < q + 1 ? nh - 1 : q + 1;   /* extrapolation degree */
        if (r > 3) r = 3;
        if (r == 0) {
            for (int i = 0; i < d; ++i) xp[i] = H[0][i] + h * F[0][i];
            cstar = 0.5;
        } else {
            double w[4];
            or_extrap_weights(r, w);
            for (int i = 0; i < d; ++i) {
                double s = 0.0;
                for (int j = 0; j <= r; ++j) s += w[j] * H[j][i];
                xp[i] = s;
            }
            cstar = 1.0;
        }

        /* psi = x_{m-1} + h sum_{i>=1} beta_i f_{m-i} */
        double psi[OR_DMAX];
        for (int i = 0; i < d; ++i) {
            double s = 0.0;
            for (int j = 1; j <= q; ++j) s += beta[j] * F[j - 1][i];
            psi[i] = H[0][i] + h * s;
        }

        double x[OR_DMAX];
        memcpy(x, r == 0 ? H[0] : xp, sizeof(double) * d);
        double c = h * beta[0];
        int conv = 0;
        for (int it = 0; it < kmax; ++it) {
            double f[OR_DMAX], rhs[OR_DMAX];
            or_rhs(model, d, p, mc, rates_fixed, x, theta, f, J);
            for (int i = 0; i < d; ++i) rhs[i] = -(x[i] - psi[i] - c * f[i]);
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) A[a * d + b] = (a == b ? 1.0 : 0.0) - c * J[a * d + b];
            memcpy(Alast, A, sizeof(double) * d * d);
            if (st) st->newton_iters++;
            if (or_lu_solve(d, A, rhs) != 0) {
                if (st) st->lu_fails++;
                for (int i = 0; i < d; ++i) x[i] = NAN;
                break;
            }
            double worst = 0.0;
            for (int i = 0; i < d; ++i) {
                x[i] += rhs[i];
                double sc = fabs(x[i]) > floor_[i] ? fabs(x[i]) : floor_[i];
                double rr = fabs(rhs[i]) / sc;
                if (rr != rr) rr = INFINITY;
                if (rr > worst) worst = rr;
            }
            if (worst <= rtol) { conv = 1; break; }
        }
        if (!conv && st) st->newton_fails++;

        if (want_lte) {
            double kap = errc / (cstar + errc);
            double e[OR_DMAX];
            for (int i = 0; i < d; ++i) e[i] = x[i] - xp[i];
            /* step 1: the Euler comparison is filtered twice */
            if (r == 0) memcpy(A, Alast, sizeof(double) * d * d);
            if (or_lu_solve(d, Alast, e) != 0 || (r == 0 && or_lu_solve(d, A, e) != 0))
                for (int i = 0; i < d; ++i) e[i] = NAN;
            for (int i = 0; i < d; ++i) {
                double ei = kap * e[i];
                gam[i] += ei * ei;
            }
        }

        /* shift the histories; f at the accepted value */
        for (int j = 4; j > 0; --j) memcpy(H[j], H[j - 1], sizeof(double) * d);
        for (int j = 3; j > 0; --j) memcpy(F[j], F[j - 1], sizeof(double) * d);
        memcpy(H[0], x, sizeof(double) * d);
        or_rhs(model, d, p, mc, rates_fixed, x, theta, F[0], NULL);
        if (nh < 5) nh++;
    }
    free(Alast);
    memcpy(x_out, H[0], sizeof(double) * d);
    if (gamma_out) memcpy(gamma_out, gam, sizeof(double) * d);
    return OR_OK;
}

/* Psi of either family: lmm 0 BDF, 1 Adams-Moulton, 2 BDF with the SDIRK start-up */
int or_psi_lmm(int lmm, int model, int d, int p, const double* mc, const double* rates_fixed,
               const double* x0, const double* theta, double h, int M, int k,
               int want_lte, double rtol, int kmax, const double* floor_,
               const double* hist, int q_hist,
               double* x_out, double* gamma_out, or_psi_stats* st)
{
    if (d < 1 || d > OR_DMAX) return OR_EINVAL;
    if (lmm == 1)
        return or_psi_am(model, d, p, mc, rates_fixed, x0, theta, h, M, k, want_lte, rtol, kmax, floor_,
                         hist, q_hist, x_out, gamma_out, st);
    if (lmm == 2)
        return or_psi_bdf(model, d, p, mc, rates_fixed, x0, theta, h, M, k, want_lte, rtol, kmax, floor_,
                          hist, q_hist, 1, x_out, gamma_out, st);
    return or_psi(model, d, p, mc, rates_fixed, x0, theta, h, M, k, want_lte, rtol, kmax, floor_,
                  hist, q_hist, x_out, gamma_out, st);
}

/* ------------------------------------------------------------------------- */
/* Likelihood pi(y | x): Gaussian, independent components, known sd sigma_i, */
/* observing x_{o_i}.  Normalising constants cancel in both weight           */
/* normalisations of Algorithm 1 (steps 3(a) and 5) and are dropped.         */
/* Non-finite states give -inf.                                              */
/* ------------------------------------------------------------------------- */
double or_loglik(int m, const int* obs, const double* y, const double* sigma, const double* x)
{
    double s = 0.0;
    for (int i = 0; i < m; ++i) {
        double v = x[obs[i]];
        if (!isfinite(v)) return -INFINITY;
        double r = (y[i] - v) / sigma[i];
        s += r * r;
    }
    return -0.5 * s;
}

/* normalised weights w = exp(l - max) / sum exp(l - max); returns the log of
 * the normaliser (-inf if every entry is -inf / NaN, then w is left zero). */
double or_normalise(long N, const double* l, double* w)
{
    double mx = -INFINITY;
    for (long n = 0; n < N; ++n) if (l[n] > mx) mx = l[n];   /* NaN compares false */
    if (!(mx > -INFINITY) || !isfinite(mx)) {
        for (long n = 0; n < N; ++n) w[n] = 0.0;
        return -INFINITY;
    }
    double s = 0.0;
    for (long n = 0; n < N; ++n) {
        double e = (l[n] > -INFINITY) ? exp(l[n] - mx) : 0.0;  /* NaN -> 0 */
        w[n] = e;
        s += e;
    }
    for (long n = 0; n < N; ++n) w[n] /= s;
    return mx + log(s);
}

/* ------------------------------------------------------------------------- */
/* Systematic resampling in exact integer arithmetic (replaces the            */
/* multinomial draw of step 3(b) with the systematic scheme).                 */
/*   q_k = floor(g_k 2^S), S = 62 - ceil(log2 N); C_k = q_1 + ... + q_k;     */
/*   T = C_N; V = floor(r T / 2^64) for a uniform word r;                     */
/* output slot i (0-based) takes the first k with C_k > floor((i T + V)/N). */
/* A particle with q_k = 0 is never chosen.                                   */
/* ------------------------------------------------------------------------- */
int or_resample_shift(long N)
{
    int c = 0;
    while ((1L << c) < N) ++c;          /* ceil(log2 N) */
    return 62 - c;
}

/* integer core: q[N] (sum T, with T*N < 2^63), offset V in [0, T) */
int or_resample_int(long N, const uint64_t* q, uint64_t V, int32_t* anc)
{
    uint64_t T = 0;
    for (long k = 0; k < N; ++k) T += q[k];
    if (T == 0 || V >= T) return OR_EDEGENERATE;
    long k = 0;
    uint64_t Ck = q[0];
    for (long i = 0; i < N; ++i) {
        uint64_t target = ((uint64_t)i * T + V) / (uint64_t)N;
        while (!(Ck > target)) { ++k; Ck += q[k]; }
        anc[i] = (int32_t)k;
    }
    return OR_OK;
}

int or_resample(long N, const double* g, uint64_t r, int32_t* anc)
{
    int S = or_resample_shift(N);
    uint64_t* q = (uint64_t*)malloc(sizeof(uint64_t) * (N > 0 ? N : 1));
    uint64_t T = 0;
    for (long k = 0; k < N; ++k) {
        double v = (g[k] > 0.0) ? floor(ldexp(g[k], S)) : 0.0;
        q[k] = (uint64_t)v;
        T += q[k];
    }
    uint64_t V = (uint64_t)(((unsigned __int128)r * T) >> 64);
    int st = or_resample_int(N, q, V, anc);
    free(q);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Multinomial resampling: the literal draw of step 3(b), each output slot   */
/* an independent draw of an index with probability g_k.  On the same       */
/* integer weights q_k as above (T = C_N): slot i has its own uniform word    */
/* r_i and takes the first k with C_k > tau_i, tau_i = floor(r_i T / 2^64),   */
/* so index k is drawn with probability q_k / T.                              */
/* ------------------------------------------------------------------------- */
int or_resample_multinomial_int(long N, const uint64_t* q, const uint64_t* r, int32_t* anc)
{
    uint64_t* Cc = (uint64_t*)malloc(sizeof(uint64_t) * (N > 0 ? N : 1));
    uint64_t T = 0;
    for (long k = 0; k < N; ++k) {
        T += q[k];
        Cc[k] = T;
    }
    if (T == 0) {
        free(Cc);
        return OR_EDEGENERATE;
    }
    for (long i = 0; i < N; ++i) {
        uint64_t tau = (uint64_t)(((unsigned __int128)r[i] * T) >> 64);
        long lo = 0, hi = N - 1;            /* first k with Cc[k] > tau */
        while (lo < hi) {
            long mid = lo + (hi - lo) / 2;
            if (Cc[mid] > tau) hi = mid;
            else lo = mid + 1;
        }
        anc[i] = (int32_t)lo;
    }
    free(Cc);
    return OR_OK;
}

/* the uniform word of output slot i at step j: Philox(seed; j, i, RESAMPLE, 0)[0] */
int or_resample_multinomial(long N, const double* g, uint64_t seed, uint64_t step, int32_t* anc)
{
    int S = or_resample_shift(N);
    uint64_t* q = (uint64_t*)malloc(sizeof(uint64_t) * (N > 0 ? N : 1));
    uint64_t* r = (uint64_t*)malloc(sizeof(uint64_t) * (N > 0 ? N : 1));
    for (long k = 0; k < N; ++k) {
        double v = (g[k] > 0.0) ? floor(ldexp(g[k], S)) : 0.0;
        q[k] = (uint64_t)v;
        uint64_t key[2] = {seed, 0}, ctr[4] = {step, (uint64_t)k, PUR_RESAMPLE, 0}, wv[4];
        or_philox4x64(ctr, key, wv);
        r[k] = wv[0];
    }
    int st = or_resample_multinomial_int(N, q, r, anc);
    free(q);
    free(r);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Weighted parameter mean and covariance (Algorithm 1 steps 1 and 6):       */
/*   mean = sum_n w_n theta_n,  C = sum_n w_n (theta_n - mean)(...)^T.       */
/* Two passes; weights are taken as given (they sum to one).                  */
/* ------------------------------------------------------------------------- */
void or_moments(long N, int p, const double* theta, const double* w, double* mean, double* cov)
{
    for (int i = 0; i < p; ++i) {
        double s = 0.0;
        for (long n = 0; n < N; ++n) s += w[n] * theta[n * p + i];
        mean[i] = s;
    }
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
            double s = 0.0;
            for (long n = 0; n < N; ++n)
                s += w[n] * (theta[n * p + i] - mean[i]) * (theta[n * p + j] - mean[j]);
            cov[i * p + j] = s;
        }
}

/* Cholesky C = L L^T (L lower, row-major).  Reading: if C is not positive   */
/* definite, retry with C + delta I, delta = 1e-10 tr(C)/p, then 10x larger,  */
/* at most five retries; then the step is degenerate.                        */
int or_cholesky(int p, const double* C, double* L, int* jitters)
{
    double tr = 0.0;
    for (int i = 0; i < p; ++i) tr += C[i * p + i];
    double delta = 0.0;
    for (int attempt = 0; attempt <= 5; ++attempt) {
        if (attempt == 1) delta = 1e-10 * tr / p;
        else if (attempt > 1) delta *= 10.0;
        int ok = 1;
        for (int i = 0; i < p * p; ++i) L[i] = 0.0;
        for (int j = 0; j < p && ok; ++j) {
            double s = C[j * p + j] + delta;
            for (int k = 0; k < j; ++k) s -= L[j * p + k] * L[j * p + k];
            if (!(s > 0.0) || !isfinite(s)) { ok = 0; break; }
            double ljj = sqrt(s);
            L[j * p + j] = ljj;
            for (int i = j + 1; i < p; ++i) {
                double t = C[i * p + j];
                for (int k = 0; k < j; ++k) t -= L[i * p + k] * L[j * p + k];
                L[i * p + j] = t / ljj;
            }
        }
        if (ok) { if (jitters) *jitters = attempt; return OR_OK; }
    }
    if (jitters) *jitters = 6;
    return OR_EDEGENERATE;
}

/* ------------------------------------------------------------------------- */
/* The filter (Algorithm 1)                                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    int model, d, p, m;
    int obs[OR_MMAX];
    const double* mc;           /* model constants (chain: V, K) */
    const double* rates_fixed;  /* chain: full rate vector */
    long N;
    uint64_t seed;
    double a;                   /* Liu-West shrinkage factor, 0 < a < 1 */
    int order, substeps;        /* BDF order k and steps per interval M */
    int kmax; double rtol;      /* Newton */
    double floor_[OR_DMAX];
    double x0[OR_DMAX];
    double prior_mean[OR_PMAX], prior_sd[OR_PMAX];
    int resampling;             /* 0 systematic (integer CDF), 1 multinomial */
    int lmm;                    /* 0 BDF, 1 Adams-Moulton, 2 BDF with SDIRK start-up */
} or_config;

typedef struct {
    uint64_t j;                 /* observations assimilated */
    double t;                   /* time of x */
    double* x;                  /* [N*d] */
    double* theta;              /* [N*p] */
    double* logw;               /* [N], normalised log-weights */
    double theta_bar[OR_PMAX];
    double C[OR_PMAX * OR_PMAX];
    double L[OR_PMAX * OR_PMAX];
} or_state;

typedef struct {
    double ess;
    double state_mean[OR_DMAX];
    long newton_iters, newton_fails, lu_fails;
    long nonfinite;             /* particles given weight zero at step 5 */
    int jitters;
    int32_t first_anc;          /* spare diagnostics */
} or_diag;

/* Step 1: initialisation.  theta_0 = prior_mean + prior_sd * z (PRIOR draws of
 * step 0), x_0 = x0 for every particle, w = 1/N, then mean, covariance and
 * the Cholesky factor used by the first proliferation. */
int or_filter_init(const or_config* cfg, double t0, or_state* s)
{
    long N = cfg->N;
    int d = cfg->d, p = cfg->p;
    if (N < 1 || d < 1 || d > OR_DMAX || p < 1 || p > OR_PMAX) return OR_EINVAL;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double z[OR_PMAX];
        or_normals(cfg->seed, 0, (uint64_t)n, PUR_PRIOR, p, z);
        for (int i = 0; i < p; ++i) s->theta[n * p + i] = cfg->prior_mean[i] + cfg->prior_sd[i] * z[i];
        for (int i = 0; i < d; ++i) s->x[n * d + i] = cfg->x0[i];
        s->logw[n] = -log((double)N);
    }
    double* w = (double*)malloc(sizeof(double) * N);
    for (long n = 0; n < N; ++n) w[n] = 1.0 / (double)N;
    or_moments(N, p, s->theta, w, s->theta_bar, s->C);
    free(w);
    int jit = 0;
    int st = or_cholesky(p, s->C, s->L, &jit);
    s->j = 0;
    s->t = t0;
    return st;
}

/* Steps 2-6 for the next observation y (m values, sd sigma) at t_next;
 * anc_in, when given, replaces the index draw of step 3(b) by these N
 * ancestors (test use: the rest of the step for another implementation's
 * draw), each in [0, N). */
static int filter_step(const or_config* cfg, or_state* s, double t_next,
                       const double* y, const double* sigma, const int32_t* anc_in, or_diag* dg)
{
    long N = cfg->N;
    int d = cfg->d, p = cfg->p, m = cfg->m;
    if (!(t_next > s->t)) return OR_EINVAL;
    for (int i = 0; i < m; ++i) if (!isfinite(y[i]) || !(sigma[i] > 0.0) || !isfinite(sigma[i])) return OR_EINVAL;
    double h = (t_next - s->t) / cfg->substeps;
    uint64_t step = s->j + 1;
    double a = cfg->a, sh = sqrt(1.0 - a * a);

    double* mshr = (double*)malloc(sizeof(double) * N * p);   /* shrunk parameters */
    double* xbar = (double*)malloc(sizeof(double) * N * d);   /* predictor states */
    double* lbar = (double*)malloc(sizeof(double) * N);       /* log pi(y | xbar) */
    double* lg   = (double*)malloc(sizeof(double) * N);
    double* g    = (double*)malloc(sizeof(double) * N);
    int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * N);
    double* xn   = (double*)malloc(sizeof(double) * N * d);
    double* thn  = (double*)malloc(sizeof(double) * N * p);
    double* lwn  = (double*)malloc(sizeof(double) * N);
    double* wn   = (double*)malloc(sizeof(double) * N);
    long it_tot = 0, fail_tot = 0, lu_tot = 0;
    int status = OR_OK;

    /* Step 2: shrink, then the predictor Psi(x_j, theta_bar_j^n, h) */
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : it_tot, fail_tot, lu_tot)
    for (long n = 0; n < N; ++n) {
        for (int i = 0; i < p; ++i) mshr[n * p + i] = a * s->theta[n * p + i] + (1.0 - a) * s->theta_bar[i];
        or_psi_stats st = {0, 0, 0};
        or_psi_lmm(cfg->lmm, cfg->model, d, p, cfg->mc, cfg->rates_fixed, s->x + n * d, mshr + n * p, h,
               cfg->substeps, cfg->order, 0, cfg->rtol, cfg->kmax, cfg->floor_, NULL, 0,
               xbar + n * d, NULL, &st);
        it_tot += st.newton_iters; fail_tot += st.newton_fails; lu_tot += st.lu_fails;
        /* Step 3(a): fitness weights g = w_j pi(y | xbar), in logs */
        lbar[n] = or_loglik(m, cfg->obs, y, sigma, xbar + n * d);
        lg[n] = s->logw[n] + lbar[n];
    }
    if (or_normalise(N, lg, g) == -INFINITY) { status = OR_EDEGENERATE; goto done; }

    /* Step 3(b): indices; systematic: one uniform word per filter and step,
     * multinomial: one per output slot */
    if (anc_in) {
        for (long n = 0; n < N; ++n) {
            if (anc_in[n] < 0 || anc_in[n] >= N) { status = OR_EINVAL; goto done; }
            anc[n] = anc_in[n];
        }
    } else if (cfg->resampling == 1) {
        if (or_resample_multinomial(N, g, cfg->seed, step, anc) != OR_OK) { status = OR_EDEGENERATE; goto done; }
    } else {
        uint64_t key[2] = {cfg->seed, 0}, ctr[4] = {step, 0, PUR_RESAMPLE, 0}, wv[4];
        or_philox4x64(ctr, key, wv);
        if (or_resample(N, g, wv[0], anc) != OR_OK) { status = OR_EDEGENERATE; goto done; }
    }

    /* Steps 3(c), 4, 5 per output slot n */
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : it_tot, fail_tot, lu_tot)
    for (long n = 0; n < N; ++n) {
        long k = anc[n];
        /* 3(c) reshuffle: x_j, xbar_{j+1}, theta_bar_j^n follow the ancestor */
        const double* xj = s->x + k * d;
        const double* mj = mshr + k * p;
        double lbar_anc = lbar[k];
        /* 4(a) proliferate: theta_{j+1} ~ N(theta_bar^n, s^2 C_j) */
        double z[OR_PMAX];
        or_normals(cfg->seed, step, (uint64_t)n, PUR_PROLIF, p, z);
        for (int i = 0; i < p; ++i) {
            double v = 0.0;
            for (int c = 0; c <= i; ++c) v += s->L[i * p + c] * z[c];
            thn[n * p + i] = mj[i] + sh * v;
        }
        /* 4(b)-(d): Gamma from the LMM error estimate, v ~ N(0, Gamma),
         * x_{j+1} = Psi(x_j, theta_{j+1}, h) + v */
        double xt[OR_DMAX], gam[OR_DMAX], zz[OR_DMAX];
        or_psi_stats st = {0, 0, 0};
        or_psi_lmm(cfg->lmm, cfg->model, d, p, cfg->mc, cfg->rates_fixed, xj, thn + n * p, h, cfg->substeps,
               cfg->order, 1, cfg->rtol, cfg->kmax, cfg->floor_, NULL, 0, xt, gam, &st);
        it_tot += st.newton_iters; fail_tot += st.newton_fails; lu_tot += st.lu_fails;
        or_normals(cfg->seed, step, (uint64_t)n, PUR_INNOV, d, zz);
        for (int i = 0; i < d; ++i) xn[n * d + i] = xt[i] + sqrt(gam[i]) * zz[i];
        /* 5: w = pi(y | x_{j+1}) / pi(y | xbar^{l_n}) */
        lwn[n] = or_loglik(m, cfg->obs, y, sigma, xn + n * d) - lbar_anc;
    }
    double lz = or_normalise(N, lwn, wn);
    if (lz == -INFINITY) { status = OR_EDEGENERATE; goto done; }

    /* 6: mean, covariance, Cholesky factor */
    double mean[OR_PMAX], cov[OR_PMAX * OR_PMAX], L[OR_PMAX * OR_PMAX];
    or_moments(N, p, thn, wn, mean, cov);
    int jit = 0;
    if (or_cholesky(p, cov, L, &jit) != OR_OK) { status = OR_EDEGENERATE; goto done; }

    /* commit */
    long nonf = 0;
    double sw2 = 0.0;
    for (long n = 0; n < N; ++n) {
        if (!(wn[n] > 0.0)) nonf += (lwn[n] == -INFINITY || lwn[n] != lwn[n]) ? 1 : 0;
        sw2 += wn[n] * wn[n];
        s->logw[n] = (wn[n] > 0.0) ? log(wn[n]) : -INFINITY;
    }
    memcpy(s->x, xn, sizeof(double) * N * d);
    memcpy(s->theta, thn, sizeof(double) * N * p);
    memcpy(s->theta_bar, mean, sizeof(double) * p);
    memcpy(s->C, cov, sizeof(double) * p * p);
    memcpy(s->L, L, sizeof(double) * p * p);
    s->j = step;
    s->t = t_next;
    if (dg) {
        dg->ess = 1.0 / sw2;
        for (int i = 0; i < d; ++i) {
            double v = 0.0;
            for (long n = 0; n < N; ++n) if (wn[n] > 0.0) v += wn[n] * xn[n * d + i];
            dg->state_mean[i] = v;
        }
        dg->newton_iters = it_tot; dg->newton_fails = fail_tot; dg->lu_fails = lu_tot;
        dg->nonfinite = nonf; dg->jitters = jit; dg->first_anc = anc[0];
    }
done:
    free(mshr); free(xbar); free(lbar); free(lg); free(g); free(anc);
    free(xn); free(thn); free(lwn); free(wn);
    return status;
}

int or_filter_step(const or_config* cfg, or_state* s, double t_next,
                   const double* y, const double* sigma, or_diag* dg)
{
    return filter_step(cfg, s, t_next, y, sigma, NULL, dg);
}

int or_filter_step_given(const or_config* cfg, or_state* s, double t_next,
                         const double* y, const double* sigma, const int32_t* anc, or_diag* dg)
{
    return filter_step(cfg, s, t_next, y, sigma, anc, dg);
}

/* diagnostic entry used by the pins: the ancestor vector and the first-stage
 * weights of one step, without committing anything (same arithmetic as
 * steps 2-3 of or_filter_step). */
int or_filter_stage1(const or_config* cfg, const or_state* s, double t_next,
                     const double* y, const double* sigma, double* g_out, int32_t* anc_out)
{
    long N = cfg->N;
    int d = cfg->d, p = cfg->p, m = cfg->m;
    double h = (t_next - s->t) / cfg->substeps;
    double a = cfg->a;
    double* lg = (double*)malloc(sizeof(double) * N);
#pragma omp parallel for schedule(dynamic, 64)
    for (long n = 0; n < N; ++n) {
        double mm[OR_PMAX], xb[OR_DMAX];
        for (int i = 0; i < p; ++i) mm[i] = a * s->theta[n * p + i] + (1.0 - a) * s->theta_bar[i];
        or_psi_lmm(cfg->lmm, cfg->model, d, p, cfg->mc, cfg->rates_fixed, s->x + n * d, mm, h, cfg->substeps,
               cfg->order, 0, cfg->rtol, cfg->kmax, cfg->floor_, NULL, 0, xb, NULL, NULL);
        lg[n] = s->logw[n] + or_loglik(m, cfg->obs, y, sigma, xb);
    }
    int st = OR_OK;
    if (or_normalise(N, lg, g_out) == -INFINITY) st = OR_EDEGENERATE;
    else if (cfg->resampling == 1) {
        st = or_resample_multinomial(N, g_out, cfg->seed, s->j + 1, anc_out);
    } else {
        uint64_t key[2] = {cfg->seed, 0}, ctr[4] = {s->j + 1, 0, PUR_RESAMPLE, 0}, wv[4];
        or_philox4x64(ctr, key, wv);
        st = or_resample(N, g_out, wv[0], anc_out);
    }
    free(lg);
    return st;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * pf_test.h -- step-level entry points of the MI355X particle-filter library,
 * exported for parity tests.  Each call runs the same device code as the
 * filter path on caller-provided DEVICE buffers and enqueues on `hip_stream`
 * (NULL = the legacy default stream); call hipStreamSynchronize (or the
 * caller's equivalent) before reading results.  Shapes are checked on the
 * host; a bad shape returns PF_EINVAL and launches nothing.
 */
#ifndef PF_TEST_H
#define PF_TEST_H

#include "pf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x64-10 (Salmon et al., SC'11) blocks: ctr [n][4], key [n][2],
 * out [n][4], all device uint64 arrays. */
pf_status pf_test_philox(uint64_t n, const uint64_t* ctr, const uint64_t* key, uint64_t* out,
                         void* hip_stream);

/* Gaussian draws of the filter's RNG map: for particle i in [0,n), `count`
 * normals of counter (step, i, purpose, block) under key (seed, 0), two
 * Box-Muller pairs per block.  out: device double [n][count]. */
pf_status pf_test_normals(uint64_t n, uint64_t seed, uint64_t step, uint64_t purpose,
                          uint32_t count, double* out, void* hip_stream);

/*
 * The integrator Psi of Algorithm 1 steps 2 and 4: n particles over one
 * interval of cfg->substeps BDF steps of size h, in cfg->precision.
 * x_in [d][n], theta [p][n] (parameters), x_out [d][n]: device doubles
 * (converted to float on entry and back on exit in FP32 mode).  With lte != 0
 * gamma [d][n] receives the innovation variance; iters (device uint64[1])
 * is incremented by the Newton iteration count (advdiff: one linear solve per
 * step, which is where Newton converges on a linear system).  Only the model,
 * dimension, integrator and Newton fields of cfg are used.
 */
pf_status pf_test_propagate(const pf_config* cfg, uint64_t n, const double* x_in,
                            const double* theta, double h, int lte, double* x_out,
                            double* gamma, uint64_t* iters, void* hip_stream);

/* Systematic resampling of normalised weights g [n] (device double) with
 * uniform word r: anc [n] (device int32) receives the ancestors.  Returns
 * PF_EDEGENERATE when every scaled weight is zero. Synchronous. */
pf_status pf_test_resample(uint64_t n, const double* g, uint64_t r, int32_t* anc,
                           void* hip_stream);

/* Multinomial resampling (the literal draw of Algorithm 1 step 3(b)) of
 * normalised weights g [n] (device double), n <= 2^20: output slot i draws
 * with its own word Philox(seed; step, i, RESAMPLE, 0)[0], as a filter's
 * step `step` does (step >= 1).  anc [n] (device int32) receives the
 * ancestors.  PF_EDEGENERATE when every scaled weight is zero; PF_EINVAL for
 * n or step out of range. Synchronous. */
pf_status pf_test_resample_multinomial(uint64_t n, const double* g, uint64_t seed, uint64_t step,
                                       int32_t* anc, void* hip_stream);

/* Algorithm 1 step 6 on given particles, through the filter's own tile
 * partials and moment pass: the mean, covariance (row-major) and Cholesky
 * factor (row-major, lower; with the jitter rule: C + delta I, delta =
 * 1e-10 tr(C)/p, times 10 up to five times) of theta [p][n] under the weights
 * exp(logw) [n] (device doubles; logw need not be normalised, -inf = weight
 * zero), and the ESS (sum w)^2 / sum w^2.  p is one of the models' parameter
 * counts: 3, 5 or 12.  mean [p], cov [p*p], chol [p*p], ess: host outputs,
 * any may be NULL.  PF_EDEGENERATE when every weight is zero or no jitter
 * makes the covariance factorable.  Synchronous. */
pf_status pf_test_moments(uint64_t n, uint32_t p, const double* theta, const double* logw, double* mean,
                          double* cov, double* chol, double* ess, void* hip_stream);

/* The three filter-based calls below run on the context's own stream: each
 * first waits for all work on the device (so buffers the caller produced on
 * any stream are ready) and returns after its own work is done. */

/* Reads the current ensemble as doubles: x [d][N], theta [p][N], logw [N]
 * (normalised log-weights); device pointers, any may be NULL.  Synchronous. */
pf_status pf_test_get_ensemble(pf_filter* f, double* x, double* theta, double* logw);

/* Overwrites the ensemble (device doubles as above; logw need not be
 * normalised) and the host-side mean, Cholesky factor (theta_bar [p],
 * L [p*p] row-major lower, host), step counter and time.  Synchronous. */
pf_status pf_test_set_ensemble(pf_filter* f, const double* x, const double* theta,
                               const double* logw, const double* theta_bar, const double* L,
                               uint64_t step, double t);

/* Ancestors of the last completed step (device int32 [N]). Synchronous. */
pf_status pf_test_last_ancestors(pf_filter* f, int32_t* anc);

#ifdef __cplusplus
}
#endif

#endif /* PF_TEST_H */

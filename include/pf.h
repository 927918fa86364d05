/*
 * pf.h -- C ABI of the MI355X particle-filter library.
 *
 * The library implements the LMM PF-SMC sampler (Arnold, Calvetti &
 * Somersalo, Sec. 2, Algorithm 1): a Liu-West auxiliary particle filter whose
 * particles carry a stiff ODE state propagated between observations by fixed
 * step BDF formulas with Newton iterations, an innovation whose variance
 * comes from the integrator's local-error estimate, likelihood weighting,
 * systematic resampling and the weighted parameter mean and covariance.
 *
 * Conventions for every call:
 *  - Pointers named in the signatures are HOST pointers unless stated.
 *    Host arrays are owned by the caller and only read (or written) during
 *    the call; the library keeps no reference to them.
 *  - Handles are owned by the library and released by the matching destroy.
 *  - Errors are returned as pf_status; pf_last_error() gives a message for
 *    the calling thread.  On any error the filter's ensemble is unchanged.
 *  - A filter is not re-entrant; different filters of one context may be
 *    driven from different threads (the context serialises submission).
 *
 * Layout of the ensemble in device memory (HBM): structure of arrays, one
 * contiguous array per state component and per parameter, padded to a
 * multiple of 256 particles (padding particles carry zero weight).  The
 * advection-diffusion field is the exception: one contiguous [d] block per
 * particle, since each particle is propagated by one workgroup.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_context pf_context;
typedef struct pf_filter pf_filter;

typedef enum {
    PF_OK = 0,
    PF_EINVAL = 1,       /* bad argument, NULL pointer, size mismatch, NaN data */
    PF_ENOMEM = 2,       /* the context's device pool cannot hold the request */
    PF_EADMIT = 3,       /* not admitted now (serving: try again when memory frees) */
    PF_EDEGENERATE = 4,  /* every weight zero or covariance not factorable: step skipped */
    PF_ENONFINITE = 5,   /* reserved */
    PF_EDEVICE = 6,      /* HIP runtime error (message in pf_last_error) */
    PF_EBUSY = 7,        /* too many steps in flight for this filter */
    PF_EORDER = 8        /* observation time not after the filter's current time */
} pf_status;

typedef enum {
    PF_MODEL_ROBERTSON = 1, /* 3 states, 3 log-rates (A->B, 2B->B+C, B+C->A+C) */
    PF_MODEL_CHAIN16 = 2,   /* 16 compartments, first 12 log-rates estimated */
    PF_MODEL_ADVDIFF = 3    /* Sec. 4: 2D periodic advection-diffusion on an nt x nt grid
                             * (d = nt^2, 3 <= nt <= 39), dU/dt = L U with
                             * L = -(k1^2 B1'B1 + k1 k3 (B1'B2 + B2'B1) + (k2^2 + k3^2) B2'B2)
                             *     + c1 B1 + c2 B2, B1 = I (x) l, B2 = l (x) I, l the periodic
                             * difference matrix of Sec. 4, grid stacked x fastest
                             * (u[iy * nt + ix]); 5 parameters (k1, k2, k3, c1, c2) used as
                             * they are (not logarithms); BDF or BDF_SDIRK only */
} pf_model;

/* Implicit LMM family of the propagation (Sec. 2: AM or BDF).  The order
 * field is the BDF order k (k steps, order k), or for AM the number of steps
 * k of the Adams-Moulton formula (order k + 1; AM1 is the trapezoidal rule;
 * AM2 and AM3 are not A-stable, so stiff models need AM1 or small steps).
 *   BDF:       each interval restarts the history (the filter carries only
 *              x_j), and step m of the interval uses order
 *              q = max(1, min(k, m - 1)): steps 1 and 2 are BDF1, BDFk is
 *              reached at step k + 1 (the interval is of order 1, 2, 2 for
 *              k = 1, 2, 3).
 *   BDF_SDIRK: the first k-1 steps of each interval instead take one step
 *              each of an L-stable, stiffly accurate SDIRK method of order k
 *              (k stages; Alexander's order-2 and order-3 methods), step k
 *              uses BDF(k-1) on the k values then available, and BDFk
 *              follows; the one lower-order step has a local error of order
 *              h^k, so the interval keeps order k.  The local-error estimate
 *              of step 4(b) of Algorithm 1 (Sec. 2; its formula is the
 *              library's own reading, the paper defers it to a companion
 *              paper) takes at those steps the ramp's comparison value and
 *              constant.  With order 1 it is plain BDF1. */
typedef enum { PF_LMM_BDF = 0, PF_LMM_AM = 1, PF_LMM_BDF_SDIRK = 2 } pf_lmm;

typedef enum {
    PF_PREC_FP64 = 0,      /* propagation (BDF + Newton + LU) in double */
    PF_PREC_FP32_PROP = 1  /* propagation and the step's normals in float; parameters, weights,
                              moments, Cholesky in double */
} pf_precision;

/* Step 3(b) index draw.  Both act on the integer weights q_k = floor(g_k 2^S),
 * S = 62 - ceil(log2 N), with T = sum q_k.
 *   SYSTEMATIC: one uniform word r per filter and step, V = floor(r T / 2^64);
 *               output slot i takes the first k with C_k > floor((i T + V)/N).
 *   MULTINOMIAL: the literal draw of Algorithm 1 step 3(b): slot i has its own
 *               word r_i = Philox(seed; step, i, RESAMPLE, 0)[0] and takes the
 *               first k with C_k > floor(r_i T / 2^64); N <= 2^20. */
typedef enum { PF_RESAMPLE_SYSTEMATIC = 0, PF_RESAMPLE_MULTINOMIAL = 1 } pf_resampling;

/*
 * Filter configuration (Algorithm 1, problem statement of Sec. 2).
 * Array fields are host pointers read during pf_create only.
 */
typedef struct {
    uint32_t struct_size;        /* sizeof(pf_config), for ABI versioning */
    pf_model model;
    uint32_t d, p, m;            /* state dim, estimated params, observed components
                                  * (m <= 4; advdiff: m <= 32) */
    const uint32_t* obs_index;   /* [m] observed state components (0-based) */
    const double* model_consts;  /* chain: [V(16), K(16)]; advdiff: [nt]; Robertson: NULL */
    uint32_t n_model_consts;     /* 32 for the chain, 1 for advdiff, 0 for Robertson */
    const double* rates_fixed;   /* chain: [16] rates; entries p..15 are the known ones */
    uint32_t n_rates_fixed;
    uint64_t n_particles;        /* N >= 1, at most 2^24 */
    uint64_t seed;               /* key of the counter-based RNG */
    double t0;                   /* time of x0 */
    const double* x0;            /* [d] initial state, the same for every particle */
    const double* prior_mean;    /* [p] Gaussian prior of the parameters (log-rates for the
                                  * kinetic models) */
    const double* prior_sd;      /* [p] */
    double shrink_a;             /* Liu-West factor, 0 < a < 1; jitter s = sqrt(1 - a^2) */
    pf_lmm lmm;
    uint32_t order;              /* BDF order k, or AM steps k; 1..3 */
    uint32_t substeps;           /* fixed steps per observation interval, 1..65536 */
    uint32_t newton_max_iter;    /* 1..64 */
    double newton_rtol;          /* stopping test max |dx_i| / max(|x_i|, floor_i) */
    const double* state_floor;   /* [d] scale floors of that test */
    pf_precision precision;
    pf_resampling resampling;    /* index draw of step 3(b) */
} pf_config;

/*
 * Caller-provided device memory for a context's pool: alloc(user, bytes,
 * stream) returns device memory of at least `bytes` bytes on the context's
 * device, aligned to 256 bytes (NULL on failure); free(user, p, stream)
 * returns it.  `stream` is the context's hipStream_t.  The library calls
 * alloc once in pf_context_create and free once in pf_context_destroy.
 */
typedef struct {
    void* (*alloc)(void* user, uint64_t bytes, void* stream);
    void (*free)(void* user, void* p, void* stream);
    void* user;
} pf_allocator;

/*
 * Context: one device, one HIP stream, a device memory pool of pool_bytes
 * (0 = 1/4 of free device memory) from which every filter's ensemble is
 * carved.  alloc: where the pool comes from (NULL, or alloc->alloc == NULL:
 * hipMalloc); the allocator is copied.  hip_stream: a hipStream_t to submit
 * on (NULL: the context creates its own, and two more on which multi-filter
 * submissions alternate, each filter's steps kept in order by events; with
 * the environment variable PF_BATCH_STREAMS=0 it uses its one stream for
 * everything).  A caller's stream is used alone.  PF_ENOMEM if the pool cannot be
 * allocated, PF_EINVAL for an allocator with only one of its functions or a
 * pool not aligned to 256 bytes.
 */
pf_status pf_context_create(int device, uint64_t pool_bytes, const pf_allocator* alloc, void* hip_stream,
                            pf_context** out);
void pf_context_destroy(pf_context* ctx);

/* Bytes of pool memory one filter with this configuration needs. */
uint64_t pf_filter_bytes(const pf_config* cfg);

/* Pool memory: bytes in use and capacity. */
pf_status pf_context_memory(pf_context* ctx, uint64_t* used, uint64_t* capacity);

/*
 * Algorithm 1, step 1: draw the ensemble from the prior (theta = mean + sd z,
 * x = x0, w = 1/N) and compute the parameter mean, covariance and Cholesky
 * factor.  Returns PF_ENOMEM when the ensemble is larger than the whole pool,
 * PF_EADMIT when the pool (or the context's table of 4096 filters) is full
 * now: try again after a filter is destroyed.  Synchronous.
 */
pf_status pf_create(pf_context* ctx, const pf_config* cfg, pf_filter** out);

/*
 * Algorithm 1, steps 2-6 for one observation y[m] with known noise sd
 * sigma[m] at time t_obs > current time.  Synchronous: returns the step's
 * status (PF_EDEGENERATE: the step was skipped, ensemble unchanged).
 */
pf_status pf_assimilate(pf_filter* f, double t_obs, const double* y, const double* sigma);

/* Asynchronous form: enqueues the step and returns a ticket (per filter,
 * increasing).  PF_EBUSY when 64 steps of this filter are already pending. */
pf_status pf_assimilate_async(pf_filter* f, double t_obs, const double* y, const double* sigma,
                              uint64_t* ticket);

/* Waits for a ticket of this filter and returns that step's status. */
pf_status pf_wait(pf_filter* f, uint64_t ticket);

/* Non-blocking: PF_EBUSY while the ticket's step is still running, otherwise
 * the step's status (the ticket is then consumed, as by pf_wait). */
pf_status pf_query(pf_filter* f, uint64_t ticket);

/*
 * Batched form: one step for `count` distinct filters of one context, as a
 * single submission.  y and sigma are [count][4] (row i uses its filter's
 * first m entries; a filter with m > 4 is rejected with PF_EINVAL).  Each
 * filter's result is identical to assimilating it alone.  tickets[count]
 * (may be NULL) receive the per-filter tickets.
 */
pf_status pf_assimilate_batch(pf_context* ctx, uint32_t count, pf_filter* const* filters,
                              const double* t_obs, const double* y, const double* sigma,
                              uint64_t* tickets);

/*
 * Posterior summary after the last completed step (waits for pending steps):
 * mean[p] and cov[p*p] (row-major) of the log-parameters (Algorithm 1 step 6),
 * optionally the weighted state mean[d], the effective sample size and the
 * number of assimilated observations.  Any output pointer may be NULL.
 */
pf_status pf_posterior(pf_filter* f, double* mean, double* cov, double* state_mean, double* ess,
                       uint64_t* step);

/* Counters since creation, written to counters[0..n) (n <= PF_STAT_COUNT):
 * Newton iterations of the predictor pass (step 2), Newton iterations of
 * the repropagation pass (step 4), integration steps that hit the Newton
 * iteration cap, particles given weight zero for a non-finite state,
 * Cholesky jitter retries, and new states x_{j+1} (after the innovation of
 * step 4(d)) with a negative component.  The kinetic models solve the Newton
 * system I - c J without pivoting, which is shown safe (every pivot >= 1)
 * for states x >= 0; the last counter tells how often a step started from
 * outside that region.  Waits for pending steps. */
enum {
    PF_STAT_NEWTON_PREDICT = 0,
    PF_STAT_NEWTON_UPDATE = 1,
    PF_STAT_NEWTON_FAILS = 2,
    PF_STAT_NONFINITE = 3,
    PF_STAT_JITTERS = 4,
    PF_STAT_NEGATIVE_STATES = 5,
    PF_STAT_COUNT = 6
};
pf_status pf_stats(pf_filter* f, uint64_t* counters, uint32_t n);

/*
 * Kernel timing for benchmarks.  With profiling on, each submission records
 * HIP events on the context's stream between its kernel groups;
 * pf_context_kernel_time waits for the recorded submissions and returns the
 * number of timed submissions and their summed milliseconds for one group:
 * PF_TIME_STEP (whole step), PF_TIME_PREDICT (step 2 and 3a kernels),
 * PF_TIME_RESAMPLE (step 3b kernels), PF_TIME_UPDATE (steps 3c-5 kernels,
 * which also form the per-tile moment sums), PF_TIME_MOMENTS (step 6: the
 * per-filter moments, Cholesky factor and commit).  Each interval lies between
 * two events on the context's stream, so it includes one dispatch gap.
 * pf_context_profile(ctx, on) clears the totals.
 */
enum { PF_TIME_STEP = 0, PF_TIME_PREDICT = 1, PF_TIME_RESAMPLE = 2, PF_TIME_UPDATE = 3, PF_TIME_MOMENTS = 4 };
pf_status pf_context_profile(pf_context* ctx, int enable);
pf_status pf_context_kernel_time(pf_context* ctx, int which, uint64_t* count, double* ms);

/* Launch-shape autotuner of the batched step (an implementation choice: it
 * changes how tiles map to workgroups, never what Algorithm 1 computes).  A
 * multi-filter submission runs three groups of launches: 0 the predictor
 * kernels, 1 the resampling kernels, 2 the update kernels.  For each group
 * and power-of-two bucket of the group's tile count, the first submissions
 * try every candidate grid (one workgroup per tile, or 16, 8, 4, 2
 * workgroups per compute unit, each looping over the tiles) twice, timed
 * with events on the context stream; the fastest is kept for the context's
 * lifetime.  Submissions on trial launch directly; a batch shape is captured
 * into a graph only once its groups are tuned.  Grids never change a
 * filter's arithmetic (fixed tiles, fixed per-tile order), so results are
 * bit-identical with tuning on or off.  Single-filter steps always run one
 * workgroup per tile; batches holding advection-diffusion filters use the
 * grids already chosen but run no trials (their own launches sit between
 * the groups).  On by default; PF_AUTOTUNE=0 in the environment at
 * context creation, or pf_context_autotune(ctx, 0), turns it off (the
 * default grid, min(tiles, 8 x CUs), is used; choices are kept and apply
 * again when it is turned back on).
 * pf_context_launch_grid waits for the submissions whose trials are not yet
 * counted, then reports the grid a multi-filter submission would launch for
 * `items` tiles in `group` now, and whether it was tuned (*tuned = 1).
 * PF_EINVAL: ctx NULL, group outside 0..2, items 0 or above 2^20. */
pf_status pf_context_autotune(pf_context* ctx, int enable);
pf_status pf_context_launch_grid(pf_context* ctx, int group, uint32_t items, uint32_t* grid, int* tuned);

/* Releases the filter's pool memory after its pending steps complete. */
void pf_destroy(pf_filter* f);

/* ------------------------------------------------------------------------
 * Serving: many filtering streams on one context with continuous batching.
 * A scheduler thread admits streams when the context's pool can hold their
 * ensembles (first come, first served), and repeatedly launches a tick: one
 * batched step (pf_assimilate_batch) that takes the oldest pending
 * observation of every admitted stream that has one.  Observations arriving
 * while ticks run join the next tick; up to max_inflight ticks are on the
 * GPU at once.  Each result is bit-identical to assimilating that stream
 * alone.  Latency of a step = pf_server_submit call -> result observed
 * complete by the scheduler.
 * ------------------------------------------------------------------------ */
typedef struct pf_server pf_server;

typedef struct {
    uint32_t struct_size;         /* sizeof(pf_server_config) */
    uint32_t max_inflight;        /* ticks on the GPU at once, >= 1 (0: 3) */
    uint32_t max_batch;           /* streams per tick, 1..4096 (0: 4096) */
    uint32_t reserved;
} pf_server_config;

typedef struct {
    uint64_t streams_opened, streams_admitted, streams_closed;
    uint64_t ticks, steps_completed, steps_skipped;   /* skipped = degenerate or out of order */
    uint64_t particle_steps;                          /* sum of N over completed steps */
    double latency_p50_ms, latency_p99_ms, latency_max_ms;
    double admit_wait_p50_ms, admit_wait_p99_ms;      /* open -> admitted */
    double mean_batch;                                /* streams per tick */
    double busy_s;                                    /* first submit -> last completion */
} pf_server_report;

pf_status pf_server_create(pf_context* ctx, const pf_server_config* cfg, pf_server** out);

/* Opens a stream with configuration cfg (copied).  It is admitted as soon as
 * the pool can hold it; observations submitted before that wait in its queue.
 * PF_ENOMEM if the ensemble could never fit the pool; PF_EINVAL for m > 4
 * (served steps are batched submissions). */
pf_status pf_server_open(pf_server* s, const pf_config* cfg, uint64_t* stream);

/* Queues an observation (y, sigma: [m], copied) at t_obs for the stream;
 * returns a per-stream ticket.  Times must increase per stream. */
pf_status pf_server_submit(pf_server* s, uint64_t stream, double t_obs, const double* y,
                           const double* sigma, uint64_t* ticket);

/* PF_EBUSY while the ticket's step is pending; otherwise the step's status
 * and (if latency_ms != NULL) its latency. */
pf_status pf_server_poll(pf_server* s, uint64_t stream, uint64_t ticket, double* latency_ms);

/* Waits until every submitted step of the stream is done, then reads its
 * posterior as pf_posterior does (for a closed stream: the posterior it had
 * when its memory was released). */
pf_status pf_server_posterior(pf_server* s, uint64_t stream, double* mean, double* cov, double* ess,
                              uint64_t* step);

/* Closes the stream: its memory returns to the pool after its submitted steps
 * complete (results stay pollable). */
pf_status pf_server_close(pf_server* s, uint64_t stream);

/* Waits until all submitted steps are complete and closed streams released. */
pf_status pf_server_drain(pf_server* s);

pf_status pf_server_stats(pf_server* s, pf_server_report* out);
void pf_server_destroy(pf_server* s);

/*
 * Systematic resampling of given weights without any allocation, for callers
 * that cannot allocate device memory (code that runs between graph captures,
 * tight serving loops, harnesses that forbid hipMalloc).  The same
 * computation and result as pf_test_resample: g [n] normalised weights
 * (device double), r the uniform word, anc [n] (device int32) receives the
 * ancestors; PF_EDEGENERATE when every scaled weight is zero.
 * Limit: n <= PF_NOALLOC_MAX_N (2^20).  Its scratch (the integer weights,
 * the tile sums and the draw's state, about 8 MiB) is one static device array
 * per GPU, held until the process ends; every call on a GPU uses the same
 * array, so calls that overlap on one GPU (other streams or threads) race:
 * serialise them.  Runs on `hip_stream` on the current device; synchronous
 * (it reads back the weights' total).  PF_EINVAL for NULL buffers or n out
 * of range; no memory is allocated, by this library or by HIP on its behalf.
 */
#define PF_NOALLOC_MAX_N (1ull << 20)
pf_status pf_resample_noalloc(uint64_t n, const double* g, uint64_t r, int32_t* anc, void* hip_stream);

const char* pf_status_str(pf_status s);
const char* pf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PF_H */

// pf_types.hpp -- data shared by the host runtime and the kernels: the
// per-filter descriptor (configuration + buffer pointers), the per-filter
// dynamic state, and the per-step submission records.
#pragma once
#include <stdint.h>

namespace pf {

constexpr int TILE = 256;      // particles per workgroup tile (4 wavefronts)
constexpr int DMAX = 16;       // largest state dimension of the kinetic models (held in registers)
constexpr int PMAX = 12;       // largest parameter dimension
constexpr int MMAX = 32;       // largest number of observed components
constexpr int MOBS_KIN = 4;    // observed components of the kinetic models
constexpr int BATCH_YSTRIDE = 4;   // row stride of y and sigma in a batched submission
// advection-diffusion: nt x nt grid values per particle, nt <= 39
constexpr int AD_NTMAX = 39;
constexpr int AD_DMAX = AD_NTMAX * AD_NTMAX;
constexpr int AD_P = 5;
constexpr int RING = 64;       // per-filter status ring (steps in flight)
// per-tile first-stage partials: tile max, sum exp, Newton iterations and
// failed solves of the predictor
constexpr int PART1_STRIDE = 4;
// counter columns at the end of each moment-partial row (summed unscaled):
// update iterations, failed solves (both kernels), non-finite weights,
// predictor iterations, states with a negative component
constexpr int NPLAIN = 5;
constexpr int SUBSTEPS_MAX = 65536;
constexpr int KMAX_MAX = 64;
constexpr int MULTI_MAX_TILES = 4096;   // multinomial draw: N <= 2^20 (tile offsets in LDS)
// moment accumulators per tile: the tile's max log-weight, s0, s00,
// sum w (theta - c), sum w (theta-c)(theta-c)^T (upper triangle), sum w x,
// and the NPLAIN counters
constexpr int NACC_MAX = 3 + PMAX + PMAX * (PMAX + 1) / 2 + DMAX + NPLAIN;

enum Status : int32_t {
    ST_OK = 0, ST_EINVAL = 1, ST_ENOMEM = 2, ST_EADMIT = 3, ST_EDEGENERATE = 4,
    ST_ENONFINITE = 5, ST_EDEVICE = 6, ST_EBUSY = 7, ST_EORDER = 8
};

enum Model : int32_t { MODEL_ROBERTSON = 1, MODEL_CHAIN16 = 2, MODEL_ADVDIFF = 3 };
enum Prec : int32_t { PREC_FP64 = 0, PREC_FP32 = 1 };

// RNG purposes: third word of the Philox counter (step, particle, purpose, block)
enum Purpose : uint64_t { PUR_PRIOR = 1, PUR_RESAMPLE = 2, PUR_PROLIF = 3, PUR_INNOV = 4 };

// Static configuration and buffers of one filter (device resident, written
// by the host at creation).
struct FilterDesc {
    int32_t model, d, p, m;
    int32_t order, substeps, kmax, prec;
    int32_t obs[MMAX];
    int32_t n, npad, ntiles, shift;     // shift: resampling scale 2^shift
    int32_t nacc, g_direct, resampling, lmm;    // resampling: 0 systematic, 1 multinomial; lmm: 0 BDF, 1 AM, 2 BDF + SDIRK start-up
    int32_t nt, pad_;                   // advection-diffusion: grid side (d = nt^2)
    uint64_t seed;
    double a, s, rtol;                  // shrink factor, jitter sqrt(1-a^2), Newton rtol
    double prior_mean[PMAX], prior_sd[PMAX];
    double x0[DMAX];
    double floor_[DMAX];
    float floor_f[DMAX];
    double mc[2 * DMAX];                // chain: V[16], K[16]
    float mc_f[2 * DMAX];
    double rates_fixed[DMAX];
    // buffers (structure of arrays, leading dimension npad)
    void* x[2];                         // [d][npad] state, float or double
    double* theta[2];                   // [p][npad] log-parameters
    double* logw[2];                    // [npad] unnormalised log-weights
    double* lbar;                       // [npad] log pi(y | predictor)
    double* lg;                         // [npad] first-stage log-weights
    uint64_t* q;                        // [npad] integer weights (multinomial: their inclusive prefix within the tile)
    int32_t* anc;                       // [npad] ancestors
    double* part1;                      // [PART1_STRIDE][ntiles] (max, sum exp, iterations, fails), by column
    uint64_t* tsum;                     // [ntiles] integer weight per tile (then offsets)
    double* part2;                      // [nacc][ntiles] moment partials and counters, by column
    // kinetic models: the step-4 normals of every output slot (P proliferation
    // rows, then D innovation rows, in the propagation precision), drawn ahead
    // of the update kernel, and per tile the step they were drawn for
    void* z;                            // [P + D][npad]
    uint64_t* ztag;                     // [ntiles]
    // advection-diffusion only (the state is too large for the inline arrays;
    // x is stored particle-major, [npad][d])
    const double* x0b;                  // [d] initial field
    double* smb;                        // [d] weighted state mean of the last committed step
    double* partx;                      // [d][ntiles] per-tile weighted state sums (scaled by the tile max)
};

// Dynamic state of one filter (device resident, updated by the kernels).
struct FilterState {
    double theta_bar[PMAX];
    double C[PMAX * PMAX];
    double L[PMAX * PMAX];
    double state_mean[DMAX];
    double ess;
    double t;                           // time of the current ensemble
    uint64_t j;                         // observations assimilated
    int32_t cur;                        // current ping-pong buffer
    int32_t status;                     // status of the step in progress / last step
    // step in progress
    double t_next;
    uint64_t step;                      // j + 1
    uint64_t T, V;                      // resampling total and offset
    uint64_t R;                         // the step's resampling word (drawn by the count pass)
    uint64_t j_run;                     // index of the last step the count pass ran
    unsigned long long newton_pred, newton_upd, newton_fails, nonfinite, jitters;
    // new states with a negative component: the kinetic models' unpivoted
    // elimination of I - c J is shown safe (every pivot >= 1) for x >= 0 only
    unsigned long long negative;
    int32_t ring[RING];                 // status by ticket % RING
};

// One filter's entry in a submitted batch.
struct StepRec {
    int32_t slot, pad;
    uint64_t seq;
    double t_next;
    double y[MMAX], sigma[MMAX];
};

// Where the step kernels find their batch (passed by value as a kernel
// argument).  A batch of one filter carries its record and a copy of its
// descriptor here (the kernels' inline form): nothing is copied ahead of the
// kernels, item i is tile i, and the descriptor fields are read from the
// kernel arguments without first looking up the slot.  Larger batches point
// at the device copy of the records and of the (entry << 16 | tile) item
// list, and read descriptors from the context's table.
struct Batch {
    const StepRec* recs;       // nullptr in the inline form
    const uint32_t* items;     // unused in the inline form
    int32_t n_items;           // tiles this launch covers
    int32_t count;             // batch entries
    StepRec one;               // inline form: the record
    FilterDesc fd;             // inline form: the filter's descriptor
};

}  // namespace pf

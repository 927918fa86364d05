// pf_runtime.hip -- host runtime behind the C ABI of include/pf.h and
// include/pf_test.h: context (device, stream, memory pool, filter table),
// filter creation (prior draw), step submission for one filter or a batch,
// tickets, posterior read-back, and the step-level test entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pf.h"
#include "../../include/pf_test.h"
#include "pf_kernels.hip"

using namespace pf;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static pf_status fail(pf_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(PF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

extern "C" const char* pf_status_str(pf_status s)
{
    switch (s) {
    case PF_OK: return "ok";
    case PF_EINVAL: return "invalid argument";
    case PF_ENOMEM: return "device pool exhausted";
    case PF_EADMIT: return "not admitted";
    case PF_EDEGENERATE: return "degenerate weights or covariance; step skipped";
    case PF_ENONFINITE: return "non-finite values";
    case PF_EDEVICE: return "HIP runtime error";
    case PF_EBUSY: return "too many steps in flight";
    case PF_EORDER: return "observation time not after the current time";
    }
    return "unknown status";
}

extern "C" const char* pf_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// device pool: one allocation, first-fit free list with coalescing
// ---------------------------------------------------------------------------
struct Pool {
    char* base = nullptr;
    uint64_t cap = 0, used = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> size

    static uint64_t align(uint64_t v) { return (v + 255) & ~uint64_t(255); }

    bool alloc(uint64_t bytes, uint64_t* off)
    {
        bytes = align(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, roff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                used += bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = align(bytes);
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// ---------------------------------------------------------------------------
// context and filter
// ---------------------------------------------------------------------------
constexpr int MAX_SLOTS = 4096;
constexpr int NSTAGE = 4;
constexpr int MAX_BATCH = 4096;
constexpr int MAX_ITEMS = 1 << 20;   // tiles per submission

struct Ticket {
    uint64_t seq;
    std::shared_ptr<hipEvent_t> ev;
    hipStream_t stream;   // the stream the step ran on
};

struct pf_filter {
    pf_context* ctx = nullptr;
    int slot = -1;
    uint64_t pool_off = 0, pool_bytes = 0;
    FilterDesc desc{};
    double t_submitted = 0.0;
    uint64_t next_seq = 1;
    std::deque<Ticket> pending;
    std::map<uint64_t, int32_t> done_status;   // tickets completed and not yet waited on
    int cls = 0;
};

struct Stage {
    char* host = nullptr;    // pinned: [recs | items] of the submission using this block
    char* dev = nullptr;
    hipEvent_t ev = nullptr;           // completion of the last submission from this block
    hipEvent_t tev[5] = {};            // timing events of that submission (profiling)
    bool timed = false;                // tev holds an uncollected timing
    hipEvent_t uev[4] = {};            // launch-shape trial: bounds of the three tuned groups
    bool trial = false;                // uev holds an uncollected trial
    int trial_key[3] = {-1, -1, -1};   // tuner key of each group (-1: not on trial)
    int trial_cand[3] = {0, 0, 0};     // candidate grid cap tried for it
};

// Launch-shape autotuner for multi-filter submissions.  Three groups of
// launches are tuned: the predictor kernels, the resampling pair and the
// update kernels.  For each group and power-of-two bucket of its tile count
// the tuner times every candidate grid cap (one workgroup per tile, or 16,
// 8, 4, 2 workgroups per compute unit looping over the tiles) TUNE_REPS times
// on real steps, then keeps the fastest (least time of its trials).  Grid
// shapes never change a filter's arithmetic (fixed tiles, fixed per-tile
// order), so tuning leaves every result bit for bit as it is.
constexpr int TUNE_NCAND = 5;
constexpr int TUNE_REPS = 2;
struct Tune {
    float best[TUNE_NCAND];
    int samples[TUNE_NCAND];
    int chosen = -1;
};

// A captured step graph for one (staging block, batch signature).
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

struct pf_context {
    int device = 0;
    bool profiling = false;
    bool use_graphs = true;
    std::vector<hipEvent_t> ev_pool;
    std::mutex ev_mu;                           // guards ev_pool
    uint64_t prof_count = 0;
    double prof_ms[5] = {0, 0, 0, 0, 0};
    std::map<std::string, GraphEntry> graphs;   // signature -> executable graph
    std::map<std::string, int> seen;            // signature -> submissions seen (capture on the 2nd)
    uint64_t use_clock = 0;
    hipStream_t stream = nullptr;
    hipStream_t init_stream = nullptr;   // filter creation runs here, beside the step stream
    // multi-filter submissions alternate between two more streams of the
    // context (when it owns its stream), so that one batch's kernels can run
    // beside the previous one's; a filter's step waits for its previous
    // step's event when that ran on another stream
    hipStream_t sub[2] = {nullptr, nullptr};
    int sub_next = 0;
    std::shared_ptr<hipEvent_t> last_ev[3];   // latest submission's event on stream, sub[0], sub[1]
    bool own_stream = false;
    Pool pool;
    FilterDesc* d_desc = nullptr;
    FilterState* d_state = nullptr;
    int32_t* h_ring = nullptr;   // pinned, mapped: [MAX_SLOTS][RING]
    int32_t* d_ring = nullptr;
    std::vector<char> slot_used;
    Stage stage[NSTAGE];
    int stage_next = 0;
    // a single filter's untimed step takes no staging block; its record is
    // built here (host memory, read only by the launch that copies it into
    // the kernel arguments)
    Stage light;
    StepRec light_rec[1];
    int grid_cap = 2048;
    int n_cu = 256;
    bool autotune = true;
    std::map<int, Tune> tune;    // (group, bucket) -> trials and choice
    pf_allocator alloc{};        // caller's allocator of the pool (alloc == NULL: hipMalloc)
    std::mutex mu;
};

static pf_status prof_collect(pf_context* ctx);

// ---------------------------------------------------------------------------
// kernel dispatch by (model, precision, order)
// ---------------------------------------------------------------------------
typedef void (*StepKernel)(Batch, const FilterDesc*, FilterState*);
typedef void (*MomentsKernel)(Batch, const FilterDesc*, FilterState*, int32_t*);

template <template <class> class Mdl, class R, int LMM, bool INL>
static StepKernel pick_predict(int order)
{
    switch (order) {
    case 1: return k_predict<Mdl<R>, R, 1, LMM, INL>;
    case 2: return k_predict<Mdl<R>, R, 2, LMM, INL>;
    default: return k_predict<Mdl<R>, R, 3, LMM, INL>;
    }
}
template <template <class> class Mdl, class R, int LMM, bool INL>
static StepKernel pick_update(int order)
{
    switch (order) {
    case 1: return k_update<Mdl<R>, R, 1, LMM, INL>;
    case 2: return k_update<Mdl<R>, R, 2, LMM, INL>;
    default: return k_update<Mdl<R>, R, 3, LMM, INL>;
    }
}
template <template <class> class Mdl, class R, bool INL>
static StepKernel predict_of(int lmm, int order)
{
    if (lmm == 1) return pick_predict<Mdl, R, 1, INL>(order);
    if (lmm == 2) return pick_predict<Mdl, R, 2, INL>(order);
    return pick_predict<Mdl, R, 0, INL>(order);
}
template <template <class> class Mdl, class R, bool INL>
static StepKernel update_of(int lmm, int order)
{
    if (lmm == 1) return pick_update<Mdl, R, 1, INL>(order);
    if (lmm == 2) return pick_update<Mdl, R, 2, INL>(order);
    return pick_update<Mdl, R, 0, INL>(order);
}
template <bool INL>
static StepKernel predict_kernel(int model, int lmm, int prec, int order)
{
    if (model == MODEL_ROBERTSON)
        return prec == PREC_FP32 ? predict_of<Robertson, float, INL>(lmm, order)
                                 : predict_of<Robertson, double, INL>(lmm, order);
    return prec == PREC_FP32 ? predict_of<Chain16, float, INL>(lmm, order)
                             : predict_of<Chain16, double, INL>(lmm, order);
}
template <bool INL>
static StepKernel update_kernel(int model, int lmm, int prec, int order)
{
    if (model == MODEL_ROBERTSON)
        return prec == PREC_FP32 ? update_of<Robertson, float, INL>(lmm, order)
                                 : update_of<Robertson, double, INL>(lmm, order);
    return prec == PREC_FP32 ? update_of<Chain16, float, INL>(lmm, order)
                             : update_of<Chain16, double, INL>(lmm, order);
}

typedef void (*InitKernel)(int, const FilterDesc*, FilterState*);
static InitKernel init_kernel(int model, int prec)
{
    if (model == MODEL_ROBERTSON)
        return prec == PREC_FP32 ? k_init<Robertson<float>, float> : k_init<Robertson<double>, double>;
    if (model == MODEL_ADVDIFF) return prec == PREC_FP32 ? k_ad_init<float> : k_ad_init<double>;
    return prec == PREC_FP32 ? k_init<Chain16<float>, float> : k_init<Chain16<double>, double>;
}
static InitKernel init_moments_kernel(int model)
{
    if (model == MODEL_ROBERTSON) return k_init_moments<Robertson<double>>;
    if (model == MODEL_ADVDIFF) return k_init_moments<AdTag>;
    return k_init_moments<Chain16<double>>;
}

// advection-diffusion kernels of one filter: workgroup shape by grid side,
// precision; LDS bytes of one particle
typedef void (*AdStepKernel)(StepRec, int, const FilterDesc*, FilterState*);
struct AdKernels {
    AdStepKernel predict, part1, update, part2;
    int wgs;
    size_t lds;
};
static AdKernels ad_kernels(const FilterDesc& d)
{
    AdKernels k;
    const bool f32 = d.prec == PREC_FP32, small = d.nt <= AdSmall::NTB;
    // the grid sides of Sec. 4 (n = 20, 40) have their own instances with the
    // transform loops unrolled; other sides run the generic ones
    if (small && d.nt == 19) {
        k.predict = f32 ? k_ad_predict<float, AdSmall, 19> : k_ad_predict<double, AdSmall, 19>;
        k.update = f32 ? k_ad_update<float, AdSmall, 19> : k_ad_update<double, AdSmall, 19>;
    } else if (small) {
        k.predict = f32 ? k_ad_predict<float, AdSmall, 0> : k_ad_predict<double, AdSmall, 0>;
        k.update = f32 ? k_ad_update<float, AdSmall, 0> : k_ad_update<double, AdSmall, 0>;
    } else if (d.nt == 39) {
        k.predict = f32 ? k_ad_predict<float, AdLarge, 39> : k_ad_predict<double, AdLarge, 39>;
        k.update = f32 ? k_ad_update<float, AdLarge, 39> : k_ad_update<double, AdLarge, 39>;
    } else {
        k.predict = f32 ? k_ad_predict<float, AdLarge, 0> : k_ad_predict<double, AdLarge, 0>;
        k.update = f32 ? k_ad_update<float, AdLarge, 0> : k_ad_update<double, AdLarge, 0>;
    }
    k.wgs = small ? AdSmall::WGS : AdLarge::WGS;
    k.part1 = k_ad_part1;
    k.part2 = f32 ? k_ad_part2<float> : k_ad_part2<double>;
    k.lds = ad_lds_bytes(d.nt, f32 ? 4 : 8);
    return k;
}

// kernel class: ((model - 1) * 3 + lmm) * 8 + precision * 4 + order
static int class_of(const FilterDesc& d) { return ((d.model - 1) * 3 + d.lmm) * 8 + d.prec * 4 + d.order; }
static void class_decode(int cls, int& model, int& lmm, int& prec, int& order)
{
    model = cls / 24 + 1;
    lmm = (cls / 8) % 3;
    prec = (cls % 8) / 4;
    order = cls % 4;
}

// ---------------------------------------------------------------------------
// configuration checks
// ---------------------------------------------------------------------------
static pf_status check_config(const pf_config* c)
{
    if (!c) return fail(PF_EINVAL, "config is NULL");
    if (c->struct_size != sizeof(pf_config)) return fail(PF_EINVAL, "pf_config.struct_size mismatch");
    if (c->model == PF_MODEL_ROBERTSON) {
        if (c->d != 3 || c->p != 3) return fail(PF_EINVAL, "Robertson needs d = 3, p = 3");
    } else if (c->model == PF_MODEL_CHAIN16) {
        if (c->d != 16 || c->p != 12) return fail(PF_EINVAL, "chain16 needs d = 16, p = 12");
        if (!c->model_consts || c->n_model_consts != 32) return fail(PF_EINVAL, "chain16 needs 32 model constants");
        if (!c->rates_fixed || c->n_rates_fixed != 16) return fail(PF_EINVAL, "chain16 needs 16 rates");
    } else if (c->model == PF_MODEL_ADVDIFF) {
        if (!c->model_consts || c->n_model_consts != 1) return fail(PF_EINVAL, "advdiff needs the grid side as its one model constant");
        const double ntd = c->model_consts[0];
        if (!(ntd >= 3.0 && ntd <= (double)AD_NTMAX) || ntd != std::floor(ntd))
            return fail(PF_EINVAL, "advdiff grid side must be an integer in 3..39");
        const uint32_t nt = (uint32_t)ntd;
        if (c->d != nt * nt || c->p != (uint32_t)AD_P) return fail(PF_EINVAL, "advdiff needs d = nt^2, p = 5");
        if (c->lmm != PF_LMM_BDF && c->lmm != PF_LMM_BDF_SDIRK) return fail(PF_EINVAL, "advdiff supports BDF and BDF_SDIRK");
    } else {
        return fail(PF_EINVAL, "unknown model");
    }
    const uint32_t mmax = c->model == PF_MODEL_ADVDIFF ? (uint32_t)MMAX : (uint32_t)MOBS_KIN;
    if (c->m < 1 || c->m > mmax || !c->obs_index)
        return fail(PF_EINVAL, "m must be 1..4 (kinetic models) or 1..32 (advdiff), with obs_index");
    for (uint32_t i = 0; i < c->m; ++i)
        if (c->obs_index[i] >= c->d) return fail(PF_EINVAL, "obs_index out of range");
    if (c->n_particles < 1 || c->n_particles > (1ull << 24)) return fail(PF_EINVAL, "n_particles must be 1..2^24");
    if (!c->x0 || !c->prior_mean || !c->prior_sd || !c->state_floor) return fail(PF_EINVAL, "NULL array in config");
    if (!(c->shrink_a > 0.0 && c->shrink_a < 1.0)) return fail(PF_EINVAL, "shrink_a must be in (0,1)");
    if (c->lmm != PF_LMM_BDF && c->lmm != PF_LMM_AM && c->lmm != PF_LMM_BDF_SDIRK)
        return fail(PF_EINVAL, "lmm must be BDF, AM or BDF_SDIRK");
    if (c->order < 1 || c->order > 3) return fail(PF_EINVAL, "order must be 1..3");
    if (c->substeps < 1 || c->substeps > SUBSTEPS_MAX) return fail(PF_EINVAL, "substeps must be 1..65536");
    if (c->newton_max_iter < 1 || c->newton_max_iter > KMAX_MAX) return fail(PF_EINVAL, "newton_max_iter must be 1..64");
    if (!(c->newton_rtol > 0.0)) return fail(PF_EINVAL, "newton_rtol must be > 0");
    if (c->precision != PF_PREC_FP64 && c->precision != PF_PREC_FP32_PROP) return fail(PF_EINVAL, "bad precision");
    if (c->resampling != PF_RESAMPLE_SYSTEMATIC && c->resampling != PF_RESAMPLE_MULTINOMIAL)
        return fail(PF_EINVAL, "bad resampling");
    if (c->resampling == PF_RESAMPLE_MULTINOMIAL && c->n_particles > (uint64_t)MULTI_MAX_TILES * TILE)
        return fail(PF_EINVAL, "multinomial resampling needs N <= 2^20");
    for (uint32_t i = 0; i < c->p; ++i)
        if (!std::isfinite(c->prior_mean[i]) || !(c->prior_sd[i] >= 0.0)) return fail(PF_EINVAL, "bad prior");
    return PF_OK;
}

static void fill_static(FilterDesc& d, const pf_config* c)
{
    std::memset(&d, 0, sizeof(d));
    d.model = c->model;
    d.d = (int)c->d;
    d.p = (int)c->p;
    d.m = (int)c->m;
    d.order = (int)c->order;
    d.substeps = (int)c->substeps;
    d.kmax = (int)c->newton_max_iter;
    d.prec = c->precision == PF_PREC_FP32_PROP ? PREC_FP32 : PREC_FP64;
    d.resampling = c->resampling == PF_RESAMPLE_MULTINOMIAL ? 1 : 0;
    // BDF1 has no start-up: it is the same propagation either way
    d.lmm = c->lmm == PF_LMM_AM ? 1 : (c->lmm == PF_LMM_BDF_SDIRK && c->order >= 2 ? 2 : 0);
    for (uint32_t i = 0; i < c->m; ++i) d.obs[i] = (int)c->obs_index[i];
    d.n = (int)c->n_particles;
    d.ntiles = (d.n + TILE - 1) / TILE;
    d.npad = d.ntiles * TILE;
    int cl = 0;
    while ((1ll << cl) < (long long)d.n) ++cl;
    d.shift = 62 - cl;
    // the advection-diffusion state mean has its own per-tile sums (partx)
    d.nacc = 3 + d.p + d.p * (d.p + 1) / 2 + (d.model == MODEL_ADVDIFF ? 0 : d.d) + NPLAIN;
    d.nt = d.model == MODEL_ADVDIFF ? (int)c->model_consts[0] : 0;
    d.seed = c->seed;
    d.a = c->shrink_a;
    d.s = std::sqrt(1.0 - c->shrink_a * c->shrink_a);
    d.rtol = c->newton_rtol;
    for (uint32_t i = 0; i < c->p; ++i) {
        d.prior_mean[i] = c->prior_mean[i];
        d.prior_sd[i] = c->prior_sd[i];
    }
    for (uint32_t i = 0; i < c->d && i < (uint32_t)DMAX; ++i) {
        d.x0[i] = c->x0[i];
        d.floor_[i] = c->state_floor[i];
        d.floor_f[i] = (float)c->state_floor[i];
    }
    for (uint32_t i = 0; i < c->n_model_consts && i < 2 * DMAX; ++i) {
        d.mc[i] = c->model_consts[i];
        d.mc_f[i] = (float)c->model_consts[i];
    }
    for (uint32_t i = 0; i < c->n_rates_fixed && i < DMAX; ++i) d.rates_fixed[i] = c->rates_fixed[i];
}

// bytes and offsets of one filter's buffers inside its pool block
struct Layout {
    uint64_t x[2], th[2], lw[2], lbar, lg, q, anc, part1, tsum, part2, z, ztag, x0b, smb, partx, total;
};
static Layout layout_of(const FilterDesc& d)
{
    Layout L{};
    const uint64_t np = (uint64_t)d.npad, rs = d.prec == PREC_FP32 ? 4 : 8;
    uint64_t o = 0;
    auto take = [&](uint64_t b) { const uint64_t r = o; o = Pool::align(o + b); return r; };
    L.x[0] = take(d.d * np * rs);
    L.x[1] = take(d.d * np * rs);
    L.th[0] = take(d.p * np * 8);
    L.th[1] = take(d.p * np * 8);
    L.lw[0] = take(np * 8);
    L.lw[1] = take(np * 8);
    L.lbar = take(np * 8);
    L.lg = take(np * 8);
    L.q = take(np * 8);
    L.anc = take(np * 4);
    L.part1 = take((uint64_t)d.ntiles * PART1_STRIDE * 8);
    L.tsum = take((uint64_t)d.ntiles * 8);
    L.part2 = take((uint64_t)d.ntiles * d.nacc * 8);
    if (d.model != MODEL_ADVDIFF) {
        L.z = take((uint64_t)(d.p + d.d) * np * rs);
        L.ztag = take((uint64_t)d.ntiles * 8);
    }
    if (d.model == MODEL_ADVDIFF) {
        L.x0b = take((uint64_t)d.d * 8);
        L.smb = take((uint64_t)d.d * 8);
        L.partx = take((uint64_t)d.d * d.ntiles * 8);
    }
    L.total = o;
    return L;
}

static void bind_buffers(FilterDesc& d, char* base, const Layout& L)
{
    d.x[0] = base + L.x[0];
    d.x[1] = base + L.x[1];
    d.theta[0] = (double*)(base + L.th[0]);
    d.theta[1] = (double*)(base + L.th[1]);
    d.logw[0] = (double*)(base + L.lw[0]);
    d.logw[1] = (double*)(base + L.lw[1]);
    d.lbar = (double*)(base + L.lbar);
    d.lg = (double*)(base + L.lg);
    d.q = (uint64_t*)(base + L.q);
    d.anc = (int32_t*)(base + L.anc);
    d.part1 = (double*)(base + L.part1);
    d.tsum = (uint64_t*)(base + L.tsum);
    d.part2 = (double*)(base + L.part2);
    d.z = nullptr;
    d.ztag = nullptr;
    if (d.model != MODEL_ADVDIFF) {
        d.z = base + L.z;
        d.ztag = (uint64_t*)(base + L.ztag);
    }
    if (d.model == MODEL_ADVDIFF) {
        d.x0b = (const double*)(base + L.x0b);
        d.smb = (double*)(base + L.smb);
        d.partx = (double*)(base + L.partx);
    }
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
// waits for every stream of the context that runs filter steps
static void sync_streams(pf_context* ctx)
{
    (void)hipStreamSynchronize(ctx->stream);
    for (hipStream_t st : ctx->sub)
        if (st) (void)hipStreamSynchronize(st);
}

extern "C" pf_status pf_context_create(int device, uint64_t pool_bytes, const pf_allocator* alloc,
                                       void* hip_stream, pf_context** out)
{
    if (!out) return fail(PF_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(PF_EINVAL, "no such device");
    HIP_TRY(hipSetDevice(device));
    auto ctx = std::make_unique<pf_context>();
    ctx->device = device;
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    HIP_TRY(hipStreamCreateWithFlags(&ctx->init_stream, hipStreamNonBlocking));
    const char* envs = std::getenv("PF_BATCH_STREAMS");   // "0": every submission on the one stream
    if (ctx->own_stream && !(envs && envs[0] == '0'))
        for (auto& st : ctx->sub) HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    if (pool_bytes == 0) {
        size_t fr = 0, tot = 0;
        HIP_TRY(hipMemGetInfo(&fr, &tot));
        pool_bytes = fr / 4;
    }
    pool_bytes = Pool::align(pool_bytes);
    void* p = nullptr;
    if (alloc && (alloc->alloc || alloc->free) && !(alloc->alloc && alloc->free))
        return fail(PF_EINVAL, "allocator needs both alloc and free");
    if (alloc && alloc->alloc) {
        ctx->alloc = *alloc;
        p = alloc->alloc(alloc->user, pool_bytes, (void*)ctx->stream);
        if (!p) return fail(PF_ENOMEM, "the caller's allocator returned no pool");
        if (((uintptr_t)p & 255) != 0) {
            alloc->free(alloc->user, p, (void*)ctx->stream);
            return fail(PF_EINVAL, "the caller's allocator returned a pool not aligned to 256 bytes");
        }
    } else if (hipMalloc(&p, pool_bytes) != hipSuccess) {
        return fail(PF_ENOMEM, "cannot allocate the device pool");
    }
    ctx->pool.base = (char*)p;
    ctx->pool.cap = pool_bytes;
    ctx->pool.free_[0] = pool_bytes;
    HIP_TRY(hipMalloc(&ctx->d_desc, sizeof(FilterDesc) * MAX_SLOTS));
    HIP_TRY(hipMalloc(&ctx->d_state, sizeof(FilterState) * MAX_SLOTS));
    HIP_TRY(hipHostMalloc(&ctx->h_ring, sizeof(int32_t) * MAX_SLOTS * RING, hipHostMallocMapped));
    HIP_TRY(hipHostGetDevicePointer((void**)&ctx->d_ring, ctx->h_ring, 0));
    ctx->slot_used.assign(MAX_SLOTS, 0);
    const size_t sbytes = sizeof(StepRec) * MAX_BATCH + sizeof(uint32_t) * MAX_ITEMS;
    for (int s = 0; s < NSTAGE; ++s) {
        HIP_TRY(hipHostMalloc(&ctx->stage[s].host, sbytes, hipHostMallocDefault));
        HIP_TRY(hipMalloc(&ctx->stage[s].dev, sbytes));
        HIP_TRY(hipEventCreateWithFlags(&ctx->stage[s].ev, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ctx->stage[s].ev, ctx->stream));
        // timing-only events: no system-scope cache flush when recorded, so
        // an interval holds the kernels and their dispatch, not a flush
        for (int i = 0; i < 5; ++i)
            HIP_TRY(hipEventCreateWithFlags(&ctx->stage[s].tev[i], hipEventDisableSystemFence));
        for (int i = 0; i < 4; ++i)
            HIP_TRY(hipEventCreateWithFlags(&ctx->stage[s].uev[i], hipEventDisableSystemFence));
    }
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    ctx->n_cu = std::max(1, prop.multiProcessorCount);
    ctx->grid_cap = std::max(256, prop.multiProcessorCount * 8);
    const char* env = std::getenv("PF_GRAPHS");
    if (env && env[0] == '0') ctx->use_graphs = false;
    const char* envt = std::getenv("PF_AUTOTUNE");
    if (envt && envt[0] == '0') ctx->autotune = false;
    *out = ctx.release();
    return PF_OK;
}

extern "C" void pf_context_destroy(pf_context* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    sync_streams(ctx);
    for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second.exec);
    for (int s = 0; s < NSTAGE; ++s) {
        for (int i = 0; i < 5; ++i) (void)hipEventDestroy(ctx->stage[s].tev[i]);
        for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ctx->stage[s].uev[i]);
        (void)hipEventDestroy(ctx->stage[s].ev);
        (void)hipHostFree(ctx->stage[s].host);
        (void)hipFree(ctx->stage[s].dev);
    }
    (void)hipHostFree(ctx->h_ring);
    (void)prof_collect(ctx);
    for (auto& e : ctx->last_ev) e.reset();   // back into the pool
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    (void)hipFree(ctx->d_desc);
    (void)hipFree(ctx->d_state);
    if (ctx->alloc.alloc) ctx->alloc.free(ctx->alloc.user, ctx->pool.base, (void*)ctx->stream);
    else (void)hipFree(ctx->pool.base);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    for (hipStream_t st : ctx->sub)
        if (st) (void)hipStreamDestroy(st);
    (void)hipStreamDestroy(ctx->init_stream);
    delete ctx;
}

extern "C" uint64_t pf_filter_bytes(const pf_config* cfg)
{
    if (check_config(cfg) != PF_OK) return 0;
    FilterDesc d;
    fill_static(d, cfg);
    return Pool::align(layout_of(d).total);
}

extern "C" pf_status pf_context_memory(pf_context* ctx, uint64_t* used, uint64_t* capacity)
{
    if (!ctx) return fail(PF_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (used) *used = ctx->pool.used;
    if (capacity) *capacity = ctx->pool.cap;
    return PF_OK;
}

static unsigned grid_for(const pf_context* ctx, int items)
{
    return (unsigned)std::max(1, std::min(items, ctx->grid_cap));
}

// candidate grid caps of the tuner: uncapped, then 16, 8, 4, 2 per CU
static int tune_cap(const pf_context* ctx, int cand)
{
    static const int per_cu[TUNE_NCAND] = {0, 16, 8, 4, 2};
    return cand == 0 ? MAX_ITEMS : per_cu[cand] * ctx->n_cu;
}
static int tune_bucket(int items)
{
    int b = 0;
    while ((1 << b) < items) ++b;
    return b;
}
static int tune_key(int group, int items) { return items > 0 ? group * 64 + tune_bucket(items) : -1; }

// the tuner's entry for a key, created on first use: candidates whose cap
// can never bind in the bucket (cap >= its largest tile count) are the same
// launch as one workgroup per tile, so they are not tried
static Tune& tune_entry(pf_context* ctx, int key)
{
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end()) return it->second;
    Tune t;
    const int top = 1 << (key % 64);
    int open = 0;
    for (int c = 0; c < TUNE_NCAND; ++c) {
        const bool same = c > 0 && tune_cap(ctx, c) >= top;
        t.best[c] = same ? INFINITY : 0.0f;
        t.samples[c] = same ? TUNE_REPS : 0;
        open += same ? 0 : 1;
    }
    if (open == 1) t.chosen = 0;
    return ctx->tune.emplace(key, t).first->second;
}


// ---------------------------------------------------------------------------
// filter creation
// ---------------------------------------------------------------------------
extern "C" pf_status pf_create(pf_context* ctx, const pf_config* cfg, pf_filter** out)
{
    if (!ctx || !out) return fail(PF_EINVAL, "NULL argument");
    *out = nullptr;
    pf_status s = check_config(cfg);
    if (s != PF_OK) return s;
    HIP_TRY(hipSetDevice(ctx->device));
    auto f = std::make_unique<pf_filter>();
    fill_static(f->desc, cfg);
    const Layout L = layout_of(f->desc);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        int slot = -1;
        for (int i = 0; i < MAX_SLOTS; ++i)
            if (!ctx->slot_used[i]) { slot = i; break; }
        if (Pool::align(L.total) > ctx->pool.cap) return fail(PF_ENOMEM, "filter larger than the device pool");
        if (slot < 0) return fail(PF_EADMIT, "filter table full");
        uint64_t off = 0;
        if (!ctx->pool.alloc(L.total, &off)) return fail(PF_EADMIT, "device pool full now");
        ctx->slot_used[slot] = 1;
        f->slot = slot;
        f->pool_off = off;
        f->pool_bytes = L.total;
    }
    f->ctx = ctx;
    f->cls = class_of(f->desc);
    bind_buffers(f->desc, ctx->pool.base + f->pool_off, L);
    FilterState st;
    std::memset(&st, 0, sizeof(st));
    st.t = cfg->t0;
    st.status = ST_OK;
    for (int i = 0; i < (int)cfg->p; ++i) st.theta_bar[i] = cfg->prior_mean[i];
    f->t_submitted = cfg->t0;
    auto cleanup = [&](pf_status e) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->pool.release(f->pool_off, f->pool_bytes);
        ctx->slot_used[f->slot] = 0;
        return e;
    };
    if (hipMemcpyAsync(ctx->d_desc + f->slot, &f->desc, sizeof(FilterDesc), hipMemcpyHostToDevice, ctx->init_stream) != hipSuccess ||
        hipMemcpyAsync(ctx->d_state + f->slot, &st, sizeof(FilterState), hipMemcpyHostToDevice, ctx->init_stream) != hipSuccess ||
        hipMemsetAsync(f->desc.anc, 0, sizeof(int32_t) * (size_t)f->desc.npad, ctx->init_stream) != hipSuccess)
        return cleanup(fail(PF_EDEVICE, "upload of filter descriptor failed"));
    if (f->desc.model == MODEL_ADVDIFF) {
        // the initial field, which is also the state mean of the prior ensemble
        const size_t b = sizeof(double) * (size_t)f->desc.d;
        if (hipMemcpyAsync((void*)f->desc.x0b, cfg->x0, b, hipMemcpyHostToDevice, ctx->init_stream) != hipSuccess ||
            hipMemcpyAsync(f->desc.smb, cfg->x0, b, hipMemcpyHostToDevice, ctx->init_stream) != hipSuccess ||
            hipStreamSynchronize(ctx->init_stream) != hipSuccess)
            return cleanup(fail(PF_EDEVICE, "upload of the initial field failed"));
    }
    const unsigned grid = grid_for(ctx, f->desc.ntiles);
    hipLaunchKernelGGL(init_kernel(f->desc.model, f->desc.prec), dim3(grid), dim3(TILE), 0, ctx->init_stream, f->slot,
                       ctx->d_desc, ctx->d_state);
    hipLaunchKernelGGL(init_moments_kernel(f->desc.model), dim3(1), dim3(TILE), 0, ctx->init_stream, f->slot,
                       ctx->d_desc, ctx->d_state);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->init_stream) != hipSuccess)
        return cleanup(fail(PF_EDEVICE, "initialisation kernel failed"));
    int32_t status = 0;
    if (hipMemcpy(&status, &ctx->d_state[f->slot].status, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return cleanup(fail(PF_EDEVICE, "status read failed"));
    if (status != ST_OK) return cleanup(fail((pf_status)status, "prior covariance not factorable"));
    *out = f.release();
    return PF_OK;
}

// ---------------------------------------------------------------------------
// profiling (events on the context stream)
// ---------------------------------------------------------------------------
static hipEvent_t pooled_event(pf_context* ctx)
{
    std::lock_guard<std::mutex> lk(ctx->ev_mu);
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    return e;
}

// accumulate the timing of the last submission from one staging block
static pf_status stage_collect(pf_context* ctx, Stage& sg)
{
    if (sg.trial) {
        HIP_TRY(hipEventSynchronize(sg.uev[3]));
        for (int g = 0; g < 3; ++g) {
            const int key = sg.trial_key[g];
            if (key < 0) continue;
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, sg.uev[g], sg.uev[g + 1]));
            Tune& t = tune_entry(ctx, key);
            if (t.chosen >= 0) continue;
            const int c = sg.trial_cand[g];
            t.best[c] = t.samples[c] == 0 ? ms : std::min(t.best[c], ms);
            t.samples[c]++;
            bool done = true;
            for (int k = 0; k < TUNE_NCAND; ++k) done = done && t.samples[k] >= TUNE_REPS;
            if (done) {
                int b = 0;
                for (int k = 1; k < TUNE_NCAND; ++k)
                    if (t.best[k] < t.best[b]) b = k;
                t.chosen = b;
            }
        }
        sg.trial = false;
    }
    if (!sg.timed) return PF_OK;
    HIP_TRY(hipEventSynchronize(sg.tev[4]));
    float ms[5];
    HIP_TRY(hipEventElapsedTime(&ms[0], sg.tev[0], sg.tev[4]));
    HIP_TRY(hipEventElapsedTime(&ms[1], sg.tev[0], sg.tev[1]));
    HIP_TRY(hipEventElapsedTime(&ms[2], sg.tev[1], sg.tev[2]));
    HIP_TRY(hipEventElapsedTime(&ms[3], sg.tev[2], sg.tev[3]));
    HIP_TRY(hipEventElapsedTime(&ms[4], sg.tev[3], sg.tev[4]));
    for (int i = 0; i < 5; ++i) ctx->prof_ms[i] += ms[i];
    ctx->prof_count++;
    sg.timed = false;
    return PF_OK;
}

static pf_status prof_collect(pf_context* ctx)
{
    for (int s = 0; s < NSTAGE; ++s) {
        pf_status st = stage_collect(ctx, ctx->stage[s]);
        if (st != PF_OK) return st;
    }
    return PF_OK;
}

extern "C" pf_status pf_context_profile(pf_context* ctx, int enable)
{
    if (!ctx) return fail(PF_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    pf_status s = prof_collect(ctx);
    if (s != PF_OK) return s;
    ctx->profiling = enable != 0;
    ctx->prof_count = 0;
    for (double& v : ctx->prof_ms) v = 0.0;
    return PF_OK;
}

extern "C" pf_status pf_context_autotune(pf_context* ctx, int enable)
{
    if (!ctx) return fail(PF_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->autotune = enable != 0;
    return PF_OK;
}

extern "C" pf_status pf_context_launch_grid(pf_context* ctx, int group, uint32_t items, uint32_t* grid, int* tuned)
{
    if (!ctx || group < 0 || group > 2 || items == 0 || items > (uint32_t)MAX_ITEMS)
        return fail(PF_EINVAL, "bad argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    pf_status s = prof_collect(ctx);   // trials of completed submissions count
    if (s != PF_OK) return s;
    const int key = tune_key(group, (int)items);
    auto it = ctx->tune.find(key);
    const bool ok = ctx->autotune && it != ctx->tune.end() && it->second.chosen >= 0;
    if (grid) *grid = (uint32_t)std::max(1, std::min((int)items, ok ? tune_cap(ctx, it->second.chosen) : ctx->grid_cap));
    if (tuned) *tuned = ok ? 1 : 0;
    return PF_OK;
}

extern "C" pf_status pf_context_kernel_time(pf_context* ctx, int which, uint64_t* count, double* ms)
{
    if (!ctx || which < 0 || which > 4) return fail(PF_EINVAL, "bad argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    pf_status s = prof_collect(ctx);
    if (s != PF_OK) return s;
    if (count) *count = ctx->prof_count;
    if (ms) *ms = ctx->prof_ms[which];
    return PF_OK;
}

// ---------------------------------------------------------------------------
// submission
// ---------------------------------------------------------------------------
static pf_status submit(pf_context* ctx, uint32_t count, pf_filter* const* fs, const double* t_obs,
                        const double* y, const double* sigma, int ystride, uint64_t* tickets)
{
    if (count == 0) return PF_OK;
    if (count > (uint32_t)MAX_BATCH) return fail(PF_EINVAL, "batch larger than 4096 filters");
    // validate everything before touching any filter
    uint64_t total_tiles = 0;
    for (uint32_t b = 0; b < count; ++b) {
        pf_filter* f = fs[b];
        if (!f || f->ctx != ctx) return fail(PF_EINVAL, "filter not of this context");
        for (uint32_t c = 0; c < b; ++c)
            if (fs[c] == f) return fail(PF_EINVAL, "a filter appears twice in one batch");
        if (!std::isfinite(t_obs[b])) return fail(PF_EINVAL, "non-finite observation time");
        if (!(t_obs[b] > f->t_submitted)) return fail(PF_EORDER, "observation time not increasing");
        if (f->desc.m > ystride) return fail(PF_EINVAL, "a batched filter observes more than 4 components");
        for (int i = 0; i < f->desc.m; ++i) {
            const double yy = y[(size_t)b * ystride + i], ss = sigma[(size_t)b * ystride + i];
            if (!std::isfinite(yy) || !std::isfinite(ss) || !(ss > 0.0))
                return fail(PF_EINVAL, "observation or sigma not finite and positive");
        }
        if (f->pending.size() >= RING) return fail(PF_EBUSY, "64 steps of this filter already pending");
        total_tiles += (uint64_t)f->desc.ntiles;
    }
    if (total_tiles > (uint64_t)MAX_ITEMS) return fail(PF_EINVAL, "batch has too many tiles");

    std::lock_guard<std::mutex> lk(ctx->mu);
    // A single filter's untimed step travels whole in the kernel arguments
    // (nothing is copied, no item list, no events of a staging block), so it
    // takes no staging block and does not wait for the submission that last
    // used one: the host can run ahead of the GPU up to the filter's ring of
    // pending steps.  Other submissions cycle through the staging blocks.
    const bool light = count == 1 && !ctx->profiling;
    // the stream of this submission: the context's own for a single filter
    // and for profiled submissions (their events bracket kernel groups),
    // else the next of the two batch streams
    hipStream_t S = ctx->stream;
    if (!light && !ctx->profiling && ctx->sub[0]) {
        S = ctx->sub[ctx->sub_next];
        ctx->sub_next ^= 1;
    }
    const int si = light ? -1 : ctx->stage_next;
    Stage& sg = light ? ctx->light : ctx->stage[si];
    if (!light) {
        ctx->stage_next = (ctx->stage_next + 1) % NSTAGE;
        HIP_TRY(hipEventSynchronize(sg.ev));   // previous use of this staging block is done
        pf_status ps = stage_collect(ctx, sg);
        if (ps != PF_OK) return ps;
    } else {
        sg.host = (char*)ctx->light_rec;
    }
    // group tiles by kernel class so each class is one contiguous list
    const size_t rec_bytes = (sizeof(StepRec) * count + 255) & ~size_t(255);
    StepRec* recs = (StepRec*)sg.host;
    uint32_t* items = (uint32_t*)(sg.host + rec_bytes);
    std::map<int, std::vector<uint32_t>> by_class;
    std::string sig = std::to_string(si) + (ctx->profiling ? "p" : "n");
    for (uint32_t b = 0; b < count; ++b) {
        pf_filter* f = fs[b];
        StepRec& r = recs[b];
        std::memset(&r, 0, sizeof(r));
        r.slot = f->slot;
        r.seq = f->next_seq;
        r.t_next = t_obs[b];
        for (int i = 0; i < f->desc.m; ++i) {
            r.y[i] = y[(size_t)b * ystride + i];
            r.sigma[i] = sigma[(size_t)b * ystride + i];
        }
        if (light) continue;   // the inline form takes tile i as item i
        auto& v = by_class[f->cls];
        for (int t = 0; t < f->desc.ntiles; ++t) v.push_back((b << 16) | (uint32_t)t);
        sig += "," + std::to_string(f->slot) + ":" + std::to_string(f->cls) + ":" + std::to_string(f->desc.ntiles);
    }
    struct Range { int cls, off, cnt; };
    std::vector<Range> ranges;
    int off = 0;
    if (light) {
        ranges.push_back({fs[0]->cls, 0, fs[0]->desc.ntiles});
        off = fs[0]->desc.ntiles;
    }
    for (auto& kv : by_class) {
        std::memcpy(items + off, kv.second.data(), kv.second.size() * sizeof(uint32_t));
        ranges.push_back({kv.first, off, (int)kv.second.size()});
        off += (int)kv.second.size();
    }
    const int n_all = off;
    const bool timed = ctx->profiling;
    // launch shapes: the tuned grid cap of each group, or a candidate on trial
    int n_kin = 0;
    for (const Range& r : ranges) {
        int model, lmm, prec, order;
        class_decode(r.cls, model, lmm, prec, order);
        if (model != MODEL_ADVDIFF) n_kin += r.cnt;
    }
    bool has_ad = false;   // advection-diffusion launches sit between the groups' events
    for (uint32_t b = 0; b < count; ++b) has_ad = has_ad || fs[b]->desc.model == MODEL_ADVDIFF;
    const int gkey[3] = {tune_key(0, n_kin), tune_key(1, n_all), tune_key(2, n_kin)};
    int gcap[3], gcand[3] = {-1, -1, -1};
    bool trial = false;
    for (int g = 0; g < 3; ++g) {
        // a single filter's step keeps one workgroup per tile (up to the cap)
        gcap[g] = ctx->grid_cap;
        if (!ctx->autotune || gkey[g] < 0 || count == 1) continue;
        Tune& t = tune_entry(ctx, gkey[g]);
        if (t.chosen >= 0) {
            gcap[g] = tune_cap(ctx, t.chosen);
            continue;
        }
        if (timed || has_ad) continue;   // trials only where the events bracket the group alone
        int c = 0;
        for (int k = 1; k < TUNE_NCAND; ++k)
            if (t.samples[k] < t.samples[c]) c = k;
        gcand[g] = c;
        gcap[g] = tune_cap(ctx, c);
        trial = true;
    }
    auto grid_of = [](int cap, int items) { return (unsigned)std::max(1, std::min(items, cap)); };
    // one filter: its record travels in the kernel arguments and nothing is
    // copied ahead of the kernels; otherwise one copy of [recs | items]
    const bool inline_rec = count == 1;
    Batch all{};
    all.count = (int32_t)count;
    all.n_items = n_all;
    if (inline_rec) {
        all.one = recs[0];
        all.fd = fs[0]->desc;
    } else {
        all.recs = (const StepRec*)sg.dev;
        all.items = (const uint32_t*)(sg.dev + rec_bytes);
    }
    auto part = [&](const Range& r) {
        Batch b = all;
        if (b.recs) b.items += r.off;
        b.n_items = r.cnt;
        return b;
    };

    MomentsKernel moments_kernel = k_moments<false, 0>;
    if (inline_rec) {
        const int mdl = fs[0]->desc.model;
        moments_kernel = mdl == MODEL_ROBERTSON ? k_moments<true, MODEL_ROBERTSON>
                         : mdl == MODEL_CHAIN16 ? k_moments<true, MODEL_CHAIN16>
                                                : k_moments<true, MODEL_ADVDIFF>;
    }
    // advection-diffusion filters: their own kernels, one launch per filter,
    // with the record in the kernel arguments (so such batches are not
    // captured into graphs)
    std::vector<uint32_t> ad_entries;
    for (uint32_t b = 0; b < count; ++b)
        if (fs[b]->desc.model == MODEL_ADVDIFF) ad_entries.push_back(b);
    auto ad_launch = [&](bool update) {
        for (uint32_t b : ad_entries) {
            const FilterDesc& d = fs[b]->desc;
            const AdKernels k = ad_kernels(d);
            const unsigned gp = (unsigned)std::min(d.n, 65535);
            // part2: one workgroup per (tile, chunk of grid points)
            const int nch = (d.d + AD_CHUNK - 1) / AD_CHUNK;
            const unsigned gt = grid_for(ctx, update ? d.ntiles * nch : d.ntiles);
            const int slot = fs[b]->slot;
            hipLaunchKernelGGL(update ? k.update : k.predict, dim3(gp), dim3(k.wgs), k.lds, S, recs[b],
                               slot, ctx->d_desc, ctx->d_state);
            hipLaunchKernelGGL(update ? k.part2 : k.part1, dim3(gt), dim3(TILE), 0, S, recs[b], slot,
                               ctx->d_desc, ctx->d_state);
        }
    };

    // the step: the copy (batches only), then the kernel groups
    auto enqueue = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        if (!inline_rec) {
            e = hipMemcpyAsync(sg.dev, sg.host, rec_bytes + sizeof(uint32_t) * n_all, hipMemcpyHostToDevice,
                               S);
            if (e != hipSuccess) return e;
        }
        if (timed && (e = hipEventRecord(sg.tev[0], S)) != hipSuccess) return e;
        if (trial && (e = hipEventRecord(sg.uev[0], S)) != hipSuccess) return e;
        for (const Range& r : ranges) {
            int model, lmm, prec, order;
            class_decode(r.cls, model, lmm, prec, order);
            if (model == MODEL_ADVDIFF) continue;
            hipLaunchKernelGGL(inline_rec ? predict_kernel<true>(model, lmm, prec, order)
                                          : predict_kernel<false>(model, lmm, prec, order),
                               dim3(grid_of(gcap[0], r.cnt)), dim3(TILE), 0,
                               S, part(r), ctx->d_desc, ctx->d_state);
        }
        if (trial && (e = hipEventRecord(sg.uev[1], S)) != hipSuccess) return e;
        ad_launch(false);
        if (timed && (e = hipEventRecord(sg.tev[1], S)) != hipSuccess) return e;
        hipLaunchKernelGGL(inline_rec ? k_count<true> : k_count<false>, dim3(grid_of(gcap[1], n_all)), dim3(TILE), 0,
                           S, all, ctx->d_desc,
                           ctx->d_state);
        // a single kinetic filter's update kernel does the systematic scatter itself
        if (!(inline_rec && fold_scatter(fs[0]->desc)))
            hipLaunchKernelGGL(inline_rec ? k_scatter<true> : k_scatter<false>, dim3(grid_of(gcap[1], n_all)),
                               dim3(TILE), 0, S, all, ctx->d_desc,
                               ctx->d_state);
        if (trial && (e = hipEventRecord(sg.uev[2], S)) != hipSuccess) return e;
        if (timed && (e = hipEventRecord(sg.tev[2], S)) != hipSuccess) return e;
        for (const Range& r : ranges) {
            int model, lmm, prec, order;
            class_decode(r.cls, model, lmm, prec, order);
            if (model == MODEL_ADVDIFF) continue;
            hipLaunchKernelGGL(inline_rec ? update_kernel<true>(model, lmm, prec, order)
                                          : update_kernel<false>(model, lmm, prec, order),
                               dim3(grid_of(gcap[2], r.cnt)), dim3(TILE), 0,
                               S, part(r), ctx->d_desc, ctx->d_state);
        }
        if (trial && (e = hipEventRecord(sg.uev[3], S)) != hipSuccess) return e;
        ad_launch(true);
        if (timed && (e = hipEventRecord(sg.tev[3], S)) != hipSuccess) return e;
        // a single kinetic filter's moment pass also draws the next step's
        // normals, in workgroups beside the one that does the moments
        const uint32_t mom_grid =
            inline_rec && fs[0]->desc.z ? 1u + (uint32_t)std::min((fs[0]->desc.ntiles + 1) / 2, ctx->grid_cap)
                                        : std::min<uint32_t>(count, (uint32_t)ctx->grid_cap);
        hipLaunchKernelGGL(moments_kernel, dim3(mom_grid), dim3(TILE), 0,
                           S, all, ctx->d_desc, ctx->d_state, ctx->d_ring);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (timed && (e = hipEventRecord(sg.tev[4], S)) != hipSuccess) return e;
        return hipSuccess;
    };

    // a filter's previous step, if still pending on another stream, comes
    // first (outside any graph capture): this stream waits for the latest
    // submission on each such stream, which follows that step
    hipStream_t const all_streams[3] = {ctx->stream, ctx->sub[0], ctx->sub[1]};
    for (int x = 0; x < 3; ++x) {
        if (!all_streams[x] || all_streams[x] == S || !ctx->last_ev[x]) continue;
        bool need = false;
        for (uint32_t b = 0; b < count && !need; ++b)
            need = !fs[b]->pending.empty() && fs[b]->pending.back().stream == all_streams[x];
        if (need) HIP_TRY(hipStreamWaitEvent(S, *ctx->last_ev[x], 0));
    }
    bool launched = false;
    // profiled submissions launch directly: their events then bracket the
    // kernels themselves.  A single filter's step launches directly too: its
    // record is in the kernel arguments, which a graph would freeze.
    // a batch shape whose launch shapes are still on trial is launched
    // directly (its events time the trial) and captured once they are chosen
    if (ctx->use_graphs && !timed && !trial && !inline_rec && ad_entries.empty()) {
        auto it = ctx->graphs.find(sig);
        if (it == ctx->graphs.end() && ++ctx->seen[sig] >= 2) {
            // a repeated batch shape: capture it once and replay it afterwards
            if (ctx->graphs.size() >= 64) {
                sync_streams(ctx);
                auto old = ctx->graphs.begin();
                for (auto g = ctx->graphs.begin(); g != ctx->graphs.end(); ++g)
                    if (g->second.last_use < old->second.last_use) old = g;
                (void)hipGraphExecDestroy(old->second.exec);
                ctx->graphs.erase(old);
            }
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(S, hipStreamCaptureModeRelaxed);
            hipError_t e2 = e == hipSuccess ? enqueue() : e;
            if (e == hipSuccess) {
                e = hipStreamEndCapture(S, &graph);
                if (e2 != hipSuccess) e = e2;
            }
            hipGraphExec_t exec = nullptr;
            if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                ctx->use_graphs = false;   // capture unsupported here: launch directly from now on
            } else {
                it = ctx->graphs.emplace(sig, GraphEntry{exec, 0}).first;
            }
        }
        if (ctx->use_graphs && it != ctx->graphs.end()) {
            it->second.last_use = ++ctx->use_clock;
            HIP_TRY(hipGraphLaunch(it->second.exec, S));
            launched = true;
        }
    }
    if (!launched) HIP_TRY(enqueue());
    if (!light) {
        sg.timed = timed;
        sg.trial = trial;
        for (int g = 0; g < 3; ++g) {
            sg.trial_key[g] = gcand[g] >= 0 ? gkey[g] : -1;
            sg.trial_cand[g] = gcand[g] >= 0 ? gcand[g] : 0;
        }
        HIP_TRY(hipEventRecord(sg.ev, S));
    }
    hipEvent_t raw = pooled_event(ctx);
    HIP_TRY(hipEventRecord(raw, S));
    auto ev = std::shared_ptr<hipEvent_t>(new hipEvent_t(raw), [ctx](hipEvent_t* e) {
        std::lock_guard<std::mutex> lk(ctx->ev_mu);
        ctx->ev_pool.push_back(*e);   // pooled; destroyed with the context
        delete e;
    });
    ctx->last_ev[S == ctx->stream ? 0 : S == ctx->sub[0] ? 1 : 2] = ev;
    for (uint32_t b = 0; b < count; ++b) {
        pf_filter* f = fs[b];
        const uint64_t seq = f->next_seq++;
        f->t_submitted = t_obs[b];
        f->pending.push_back({seq, ev, S});
        if (tickets) tickets[b] = seq;
    }
    return PF_OK;
}

// completes every pending ticket up to and including `upto`
static pf_status drain(pf_filter* f, uint64_t upto)
{
    while (!f->pending.empty() && f->pending.front().seq <= upto) {
        Ticket t = f->pending.front();
        HIP_TRY(hipEventSynchronize(*t.ev));
        f->done_status[t.seq] = f->ctx->h_ring[(size_t)f->slot * RING + t.seq % RING];
        f->pending.pop_front();
    }
    return PF_OK;
}

extern "C" pf_status pf_assimilate_async(pf_filter* f, double t_obs, const double* y, const double* sigma,
                                         uint64_t* ticket)
{
    if (!f || !y || !sigma) return fail(PF_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(f->ctx->device));
    return submit(f->ctx, 1, &f, &t_obs, y, sigma, MMAX, ticket);   // y, sigma: [m]
}

extern "C" pf_status pf_wait(pf_filter* f, uint64_t ticket)
{
    if (!f) return fail(PF_EINVAL, "NULL filter");
    if (ticket == 0 || ticket >= f->next_seq) return fail(PF_EINVAL, "unknown ticket");
    HIP_TRY(hipSetDevice(f->ctx->device));
    pf_status s = drain(f, ticket);
    if (s != PF_OK) return s;
    auto it = f->done_status.find(ticket);
    if (it == f->done_status.end()) return fail(PF_EINVAL, "ticket already waited on");
    const pf_status st = (pf_status)it->second;
    f->done_status.erase(it);
    if (st != PF_OK) g_last_error = pf_status_str(st);
    return st;
}

extern "C" pf_status pf_query(pf_filter* f, uint64_t ticket)
{
    if (!f) return fail(PF_EINVAL, "NULL filter");
    if (ticket == 0 || ticket >= f->next_seq) return fail(PF_EINVAL, "unknown ticket");
    HIP_TRY(hipSetDevice(f->ctx->device));
    // complete every ticket up to this one whose event has fired
    while (!f->pending.empty() && f->pending.front().seq <= ticket) {
        const hipError_t q = hipEventQuery(*f->pending.front().ev);
        if (q == hipErrorNotReady) return PF_EBUSY;
        if (q != hipSuccess) return fail(PF_EDEVICE, std::string("hipEventQuery: ") + hipGetErrorString(q));
        Ticket t = f->pending.front();
        f->done_status[t.seq] = f->ctx->h_ring[(size_t)f->slot * RING + t.seq % RING];
        f->pending.pop_front();
    }
    auto it = f->done_status.find(ticket);
    if (it == f->done_status.end()) return fail(PF_EINVAL, "ticket already consumed");
    const pf_status st = (pf_status)it->second;
    f->done_status.erase(it);
    return st;
}

extern "C" pf_status pf_assimilate(pf_filter* f, double t_obs, const double* y, const double* sigma)
{
    uint64_t t = 0;
    pf_status s = pf_assimilate_async(f, t_obs, y, sigma, &t);
    if (s != PF_OK) return s;
    return pf_wait(f, t);
}

extern "C" pf_status pf_assimilate_batch(pf_context* ctx, uint32_t count, pf_filter* const* filters,
                                         const double* t_obs, const double* y, const double* sigma,
                                         uint64_t* tickets)
{
    if (!ctx || (count && (!filters || !t_obs || !y || !sigma))) return fail(PF_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(ctx->device));
    return submit(ctx, count, filters, t_obs, y, sigma, BATCH_YSTRIDE, tickets);
}

static pf_status read_state(pf_filter* f, FilterState* st)
{
    HIP_TRY(hipSetDevice(f->ctx->device));
    pf_status s = drain(f, f->next_seq - 1);
    if (s != PF_OK) return s;
    // drain has waited for this filter's steps (on whichever stream they
    // ran); the copy runs on the context's stream
    HIP_TRY(hipMemcpyAsync(st, f->ctx->d_state + f->slot, sizeof(FilterState), hipMemcpyDeviceToHost,
                           f->ctx->stream));
    HIP_TRY(hipStreamSynchronize(f->ctx->stream));
    return PF_OK;
}

extern "C" pf_status pf_posterior(pf_filter* f, double* mean, double* cov, double* state_mean, double* ess,
                                  uint64_t* step)
{
    if (!f) return fail(PF_EINVAL, "NULL filter");
    FilterState st;
    pf_status s = read_state(f, &st);
    if (s != PF_OK) return s;
    const int p = f->desc.p, d = f->desc.d;
    if (mean) for (int i = 0; i < p; ++i) mean[i] = st.theta_bar[i];
    if (cov) for (int i = 0; i < p * p; ++i) cov[i] = st.C[i];
    if (state_mean) {
        if (f->desc.model == MODEL_ADVDIFF) {
            // read on the context stream, after the filter's last step
            HIP_TRY(hipMemcpyAsync(state_mean, f->desc.smb, sizeof(double) * d, hipMemcpyDeviceToHost, f->ctx->stream));
            HIP_TRY(hipStreamSynchronize(f->ctx->stream));
        } else {
            for (int i = 0; i < d; ++i) state_mean[i] = st.state_mean[i];
        }
    }
    if (ess) *ess = st.ess;
    if (step) *step = st.j;
    return PF_OK;
}

extern "C" pf_status pf_stats(pf_filter* f, uint64_t* counters, uint32_t n)
{
    if (!f || (n && !counters)) return fail(PF_EINVAL, "NULL argument");
    if (n > PF_STAT_COUNT) return fail(PF_EINVAL, "n larger than PF_STAT_COUNT");
    FilterState st;
    pf_status s = read_state(f, &st);
    if (s != PF_OK) return s;
    const uint64_t v[PF_STAT_COUNT] = {st.newton_pred, st.newton_upd, st.newton_fails, st.nonfinite, st.jitters,
                                       st.negative};
    for (uint32_t i = 0; i < n; ++i) counters[i] = v[i];
    return PF_OK;
}

extern "C" void pf_destroy(pf_filter* f)
{
    if (!f) return;
    pf_context* ctx = f->ctx;
    (void)hipSetDevice(ctx->device);
    // every kernel that touches this filter's memory belongs to one of its
    // tickets: once they are complete the memory can be reused
    (void)drain(f, f->next_seq - 1);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->pool.release(f->pool_off, f->pool_bytes);
        ctx->slot_used[f->slot] = 0;
    }
    delete f;
}

// ---------------------------------------------------------------------------
// test-only entry points
// ---------------------------------------------------------------------------
extern "C" pf_status pf_test_philox(uint64_t n, const uint64_t* ctr, const uint64_t* key, uint64_t* out,
                                    void* hip_stream)
{
    if (!ctr || !key || !out) return fail(PF_EINVAL, "NULL argument");
    if (n == 0) return PF_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_test_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, ctr, key, out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return PF_OK;
}

extern "C" pf_status pf_test_normals(uint64_t n, uint64_t seed, uint64_t step, uint64_t purpose, uint32_t count,
                                     double* out, void* hip_stream)
{
    if (!out) return fail(PF_EINVAL, "NULL argument");
    if (n == 0) return PF_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    switch (count) {
    case 1: hipLaunchKernelGGL(k_test_normals<1>, g, b, 0, s, n, seed, step, purpose, out); break;
    case 2: hipLaunchKernelGGL(k_test_normals<2>, g, b, 0, s, n, seed, step, purpose, out); break;
    case 3: hipLaunchKernelGGL(k_test_normals<3>, g, b, 0, s, n, seed, step, purpose, out); break;
    case 4: hipLaunchKernelGGL(k_test_normals<4>, g, b, 0, s, n, seed, step, purpose, out); break;
    case 5: hipLaunchKernelGGL(k_test_normals<5>, g, b, 0, s, n, seed, step, purpose, out); break;
    case 12: hipLaunchKernelGGL(k_test_normals<12>, g, b, 0, s, n, seed, step, purpose, out); break;
    case 16: hipLaunchKernelGGL(k_test_normals<16>, g, b, 0, s, n, seed, step, purpose, out); break;
    default: return fail(PF_EINVAL, "count must be one of 1,2,3,4,5,12,16");
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return PF_OK;
}

typedef void (*PropKernel)(const FilterDesc*, uint64_t, const double*, const double*, double, double*, double*,
                           unsigned long long*);

template <template <class> class Mdl, class R, bool LTE, int LMM>
static PropKernel pick_prop_lmm(int order)
{
    switch (order) {
    case 1: return k_test_propagate<Mdl<R>, R, 1, LTE, LMM>;
    case 2: return k_test_propagate<Mdl<R>, R, 2, LTE, LMM>;
    default: return k_test_propagate<Mdl<R>, R, 3, LTE, LMM>;
    }
}
template <template <class> class Mdl, class R, bool LTE>
static PropKernel pick_prop(int lmm, int order)
{
    if (lmm == 1) return pick_prop_lmm<Mdl, R, LTE, 1>(order);
    if (lmm == 2) return pick_prop_lmm<Mdl, R, LTE, 2>(order);
    return pick_prop_lmm<Mdl, R, LTE, 0>(order);
}

extern "C" pf_status pf_test_propagate(const pf_config* cfg, uint64_t n, const double* x_in, const double* theta,
                                       double h, int lte, double* x_out, double* gamma, uint64_t* iters,
                                       void* hip_stream)
{
    pf_status s = check_config(cfg);
    if (s != PF_OK) return s;
    if (!x_in || !theta || !x_out || (lte && !gamma)) return fail(PF_EINVAL, "NULL buffer");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(PF_EINVAL, "h must be positive");
    if (n == 0) return PF_OK;
    FilterDesc d;
    fill_static(d, cfg);
    hipStream_t st = (hipStream_t)hip_stream;
    FilterDesc* dd = nullptr;
    HIP_TRY(hipMalloc(&dd, sizeof(FilterDesc)));
    hipError_t e = hipMemcpyAsync(dd, &d, sizeof(FilterDesc), hipMemcpyHostToDevice, st);
    PropKernel k;
    const bool f32 = d.prec == PREC_FP32;
    if (d.model == MODEL_ADVDIFF) {
        const bool small = d.nt <= AdSmall::NTB;
        PropKernel ka;
        if (small && d.nt == 19)
            ka = f32 ? (lte ? k_ad_test_propagate<float, AdSmall, true, 19> : k_ad_test_propagate<float, AdSmall, false, 19>)
                     : (lte ? k_ad_test_propagate<double, AdSmall, true, 19> : k_ad_test_propagate<double, AdSmall, false, 19>);
        else if (small)
            ka = f32 ? (lte ? k_ad_test_propagate<float, AdSmall, true, 0> : k_ad_test_propagate<float, AdSmall, false, 0>)
                     : (lte ? k_ad_test_propagate<double, AdSmall, true, 0> : k_ad_test_propagate<double, AdSmall, false, 0>);
        else if (d.nt == 39)
            ka = f32 ? (lte ? k_ad_test_propagate<float, AdLarge, true, 39> : k_ad_test_propagate<float, AdLarge, false, 39>)
                     : (lte ? k_ad_test_propagate<double, AdLarge, true, 39> : k_ad_test_propagate<double, AdLarge, false, 39>);
        else
            ka = f32 ? (lte ? k_ad_test_propagate<float, AdLarge, true, 0> : k_ad_test_propagate<float, AdLarge, false, 0>)
                     : (lte ? k_ad_test_propagate<double, AdLarge, true, 0> : k_ad_test_propagate<double, AdLarge, false, 0>);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(ka, dim3((unsigned)std::min<uint64_t>(n, 65535)), dim3(small ? AdSmall::WGS : AdLarge::WGS),
                               ad_lds_bytes(d.nt, f32 ? 4 : 8), st, dd, n, x_in, theta, h, x_out, lte ? gamma : nullptr,
                               (unsigned long long*)iters);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(dd);
        if (e != hipSuccess) return fail(PF_EDEVICE, std::string("propagate: ") + hipGetErrorString(e));
        return PF_OK;
    }
    if (d.model == MODEL_ROBERTSON)
        k = f32 ? (lte ? pick_prop<Robertson, float, true>(d.lmm, d.order) : pick_prop<Robertson, float, false>(d.lmm, d.order))
                : (lte ? pick_prop<Robertson, double, true>(d.lmm, d.order) : pick_prop<Robertson, double, false>(d.lmm, d.order));
    else
        k = f32 ? (lte ? pick_prop<Chain16, float, true>(d.lmm, d.order) : pick_prop<Chain16, float, false>(d.lmm, d.order))
                : (lte ? pick_prop<Chain16, double, true>(d.lmm, d.order) : pick_prop<Chain16, double, false>(d.lmm, d.order));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k, dim3((unsigned)((n + TILE - 1) / TILE)), dim3(TILE), 0, st, dd, n, x_in, theta, h, x_out,
                           lte ? gamma : nullptr, (unsigned long long*)iters);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dd);
    if (e != hipSuccess) return fail(PF_EDEVICE, std::string("propagate: ") + hipGetErrorString(e));
    return PF_OK;
}

// both index draws through the filter's own kernels (k_count, k_scatter) on
// weights given directly; systematic: r is the uniform word, multinomial: the
// words come from (seed, step) as in a filter step
static pf_status test_resample(uint64_t n, const double* g, int multinomial, uint64_t r, uint64_t seed,
                               uint64_t step, int32_t* anc, void* hip_stream)
{
    if (!g || !anc) return fail(PF_EINVAL, "NULL buffer");
    if (n == 0 || n > (1ull << 24)) return fail(PF_EINVAL, "n must be 1..2^24");
    if (multinomial && (n > (uint64_t)MULTI_MAX_TILES * TILE || step == 0))
        return fail(PF_EINVAL, "multinomial: n must be 1..2^20 and step >= 1");
    hipStream_t st = (hipStream_t)hip_stream;
    FilterDesc d;
    std::memset(&d, 0, sizeof(d));
    d.n = (int)n;
    d.ntiles = (d.n + TILE - 1) / TILE;
    d.npad = d.ntiles * TILE;
    int cl = 0;
    while ((1ll << cl) < (long long)d.n) ++cl;
    d.shift = 62 - cl;
    d.g_direct = 1;
    d.resampling = multinomial ? 1 : 0;
    d.seed = seed;
    // scratch: desc, state, rec, items, q, tsum, done
    const size_t nb = sizeof(FilterDesc) + sizeof(FilterState) + sizeof(StepRec) + 4 * (size_t)d.ntiles +
                      8 * (size_t)d.npad + 8 * (size_t)d.ntiles + 6 * 256;
    char* buf = nullptr;
    HIP_TRY(hipMalloc(&buf, nb));
    size_t o = 0;
    auto take = [&](size_t b) { char* p = buf + o; o = (o + b + 255) & ~size_t(255); return p; };
    FilterDesc* dd = (FilterDesc*)take(sizeof(FilterDesc));
    FilterState* ds = (FilterState*)take(sizeof(FilterState));
    StepRec* dr = (StepRec*)take(sizeof(StepRec));
    uint32_t* di = (uint32_t*)take(4 * (size_t)d.ntiles);
    d.q = (uint64_t*)take(8 * (size_t)d.npad);
    d.tsum = (uint64_t*)take(8 * (size_t)d.ntiles);
    d.lg = const_cast<double*>(g);
    d.anc = anc;
    FilterState hs;
    std::memset(&hs, 0, sizeof(hs));
    hs.status = ST_OK;
    hs.V = r;
    hs.j = multinomial ? step - 1 : 0;
    StepRec rec;
    std::memset(&rec, 0, sizeof(rec));
    std::vector<uint32_t> items(d.ntiles);
    for (int t = 0; t < d.ntiles; ++t) items[t] = (uint32_t)t;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(dd, &d, sizeof(d), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ds, &hs, sizeof(hs), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dr, &rec, sizeof(rec), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(di, items.data(), 4 * items.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        const unsigned grid = (unsigned)std::min(d.ntiles, 2048);
        Batch bt{};
        bt.recs = dr;
        bt.items = di;
        bt.n_items = d.ntiles;
        bt.count = 1;
        hipLaunchKernelGGL(k_count<false>, dim3(grid), dim3(TILE), 0, st, bt, dd, ds);
        hipLaunchKernelGGL(k_scatter<false>, dim3(grid), dim3(TILE), 0, st, bt, dd, ds);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hs, ds, sizeof(hs), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(PF_EDEVICE, std::string("resample: ") + hipGetErrorString(e));
    if (hs.T == 0) return fail(PF_EDEGENERATE, "all scaled weights are zero");
    return PF_OK;
}

extern "C" pf_status pf_test_resample(uint64_t n, const double* g, uint64_t r, int32_t* anc, void* hip_stream)
{
    return test_resample(n, g, 0, r, 0, 0, anc, hip_stream);
}

extern "C" pf_status pf_test_resample_multinomial(uint64_t n, const double* g, uint64_t seed, uint64_t step,
                                                  int32_t* anc, void* hip_stream)
{
    return test_resample(n, g, 1, 0, seed, step, anc, hip_stream);
}

// ---------------------------------------------------------------------------
// systematic resampling without allocation: the draw's state, the integer
// weights and the tile sums live in one static device array; the descriptor
// and the record travel by value in the kernels' inline batch form
// ---------------------------------------------------------------------------
namespace pf {
constexpr uint64_t NOALLOC_MAX_N = PF_NOALLOC_MAX_N;
constexpr size_t NOALLOC_Q_OFF = 256 * ((sizeof(FilterState) + 255) / 256);
constexpr size_t NOALLOC_TSUM_OFF = NOALLOC_Q_OFF + 8 * NOALLOC_MAX_N;
constexpr size_t NOALLOC_BYTES = NOALLOC_TSUM_OFF + 8 * (NOALLOC_MAX_N / TILE);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// the draw's state: zero except the caller's uniform word (the count pass
// takes it from V in the given-weights form)
__global__ __launch_bounds__(TILE) void k_noalloc_state(FilterState* st, uint64_t r)
{
    uint64_t* w = (uint64_t*)st;
    for (size_t i = threadIdx.x; i < sizeof(FilterState) / 8; i += TILE) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        st->status = ST_OK;
        st->V = r;
    }
}
}  // namespace pf

// device address of `scratch` on each device, looked up once per device with
// that device current (the array's name is not a device address in host code)
static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[64];

static pf_status noalloc_scratch(char** out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(PF_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PF_EDEVICE, "no device address for the static scratch");
        g_noalloc_ptr[dev] = p;
    }
    *out = (char*)g_noalloc_ptr[dev];
    return PF_OK;
}

extern "C" pf_status pf_resample_noalloc(uint64_t n, const double* g, uint64_t r, int32_t* anc, void* hip_stream)
{
    if (!g || !anc) return fail(PF_EINVAL, "NULL buffer");
    if (n == 0 || n > NOALLOC_MAX_N) return fail(PF_EINVAL, "n must be 1..2^20 (the size of the static scratch)");
    char* base = nullptr;
    const pf_status ps = noalloc_scratch(&base);
    if (ps != PF_OK) return ps;
    hipStream_t st = (hipStream_t)hip_stream;
    Batch bt;
    std::memset(&bt, 0, sizeof(bt));
    FilterDesc& d = bt.fd;
    d.n = (int)n;
    d.ntiles = (d.n + TILE - 1) / TILE;
    d.npad = d.ntiles * TILE;
    int cl = 0;
    while ((1ll << cl) < (long long)d.n) ++cl;
    d.shift = 62 - cl;
    d.g_direct = 1;
    d.resampling = 0;
    d.q = (uint64_t*)(base + NOALLOC_Q_OFF);
    d.tsum = (uint64_t*)(base + NOALLOC_TSUM_OFF);
    d.lg = const_cast<double*>(g);
    d.anc = anc;
    bt.n_items = d.ntiles;
    bt.count = 1;
    FilterState* ds = (FilterState*)base;
    const unsigned grid = (unsigned)std::min(d.ntiles, 2048);
    hipLaunchKernelGGL(k_noalloc_state, dim3(1), dim3(TILE), 0, st, ds, r);
    hipLaunchKernelGGL(k_count<true>, dim3(grid), dim3(TILE), 0, st, bt, (const FilterDesc*)nullptr, ds);
    hipLaunchKernelGGL(k_scatter<true>, dim3(grid), dim3(TILE), 0, st, bt, (const FilterDesc*)nullptr, ds);
    hipError_t e = hipGetLastError();
    uint64_t T = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&T, &ds->T, sizeof(T), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(PF_EDEVICE, std::string("resample: ") + hipGetErrorString(e));
    if (T == 0) return fail(PF_EDEGENERATE, "all scaled weights are zero");
    return PF_OK;
}

namespace pf {
template <class R>
__global__ void k_test_get(const FilterDesc* descs, const FilterState* states, int slot, double* x, double* th,
                           double* lw)
{
    const FilterDesc& fd = descs[slot];
    const int cur = states[slot].cur;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= fd.n) return;
    const R* xb = (const R*)fd.x[cur];
    // advection-diffusion fields are stored particle-major
    const bool pm = fd.model == MODEL_ADVDIFF;
    if (x)
        for (int i = 0; i < fd.d; ++i)
            x[(size_t)i * fd.n + n] = (double)xb[pm ? (size_t)n * fd.d + i : (size_t)i * fd.npad + n];
    if (th) for (int i = 0; i < fd.p; ++i) th[(size_t)i * fd.n + n] = fd.theta[cur][(size_t)i * fd.npad + n];
    if (lw) lw[n] = fd.logw[cur][n];
}
template <class R>
__global__ void k_test_set(const FilterDesc* descs, const FilterState* states, int slot, const double* x,
                           const double* th, const double* lw)
{
    const FilterDesc& fd = descs[slot];
    const int cur = states[slot].cur;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= fd.n) return;
    R* xb = (R*)fd.x[cur];
    const bool pm = fd.model == MODEL_ADVDIFF;
    for (int i = 0; i < fd.d; ++i) xb[pm ? (size_t)n * fd.d + i : (size_t)i * fd.npad + n] = (R)x[(size_t)i * fd.n + n];
    for (int i = 0; i < fd.p; ++i) fd.theta[cur][(size_t)i * fd.npad + n] = th[(size_t)i * fd.n + n];
    fd.logw[cur][n] = lw[n];
}
}  // namespace pf

namespace pf {
// step 6 on given particles: tile partials of theta [p][n] under exp(logw),
// shift zero (the descriptor's prior mean is zero), then the moment pass
template <int P>
__global__ __launch_bounds__(TILE) void k_test_tile_moments(const FilterDesc* fdp, const double* theta,
                                                           const double* logw)
{
    __shared__ double sh[TILE];
    const FilterDesc& fd = *fdp;
    for (int tile = blockIdx.x; tile < fd.ntiles; tile += gridDim.x) {
        const int n = tile * TILE + threadIdx.x;
        const bool valid = n < fd.n;
        double th[P];
#pragma unroll
        for (int i = 0; i < P; ++i) th[i] = valid ? theta[(size_t)i * fd.n + n] : 0.0;
        const double l = valid ? logw[n] : -INFINITY;
        tile_moments<double, P, 0>(l, valid, th, nullptr, fd.prior_mean, 0, nullptr, fd.part2 + tile, fd.ntiles,
                                   sh);
    }
}
template <int P>
__global__ __launch_bounds__(TILE) void k_test_moments_finish(const FilterDesc* fdp, FilterState* st)
{
    __shared__ double sh[TILE];
    __shared__ double tot[NACC_MAX];
    const FilterDesc& fd = *fdp;
    const MomPre pre = mom_prefetch<P>(*st);
    moments_combine<P, 0>(fd, tot, sh);
    const int32_t status = moments_finish<P, 0>(fd, tot, pre, *st, false, pre.t);
    if (threadIdx.x == 0) st->status = status;
}
}  // namespace pf

extern "C" pf_status pf_test_moments(uint64_t n, uint32_t p, const double* theta, const double* logw, double* mean,
                                     double* cov, double* chol, double* ess, void* hip_stream)
{
    if (!theta || !logw) return fail(PF_EINVAL, "NULL buffer");
    if (n == 0 || n > (1ull << 24)) return fail(PF_EINVAL, "n must be 1..2^24");
    if (p != 3 && p != 5 && p != 12) return fail(PF_EINVAL, "p must be 3, 5 or 12");
    hipStream_t st = (hipStream_t)hip_stream;
    FilterDesc d;
    std::memset(&d, 0, sizeof(d));
    d.n = (int)n;
    d.p = (int)p;
    d.ntiles = (d.n + TILE - 1) / TILE;
    d.npad = d.ntiles * TILE;
    d.nacc = 3 + d.p + d.p * (d.p + 1) / 2 + NPLAIN;
    char* buf = nullptr;
    const size_t part_bytes = sizeof(double) * (size_t)d.nacc * d.ntiles;
    HIP_TRY(hipMalloc(&buf, 512 + sizeof(FilterDesc) + sizeof(FilterState) + part_bytes));
    FilterDesc* dd = (FilterDesc*)buf;
    FilterState* ds = (FilterState*)(buf + ((sizeof(FilterDesc) + 255) & ~size_t(255)));
    d.part2 = (double*)((char*)ds + ((sizeof(FilterState) + 255) & ~size_t(255)));
    FilterState hs;
    std::memset(&hs, 0, sizeof(hs));
    hipError_t e = hipMemcpyAsync(dd, &d, sizeof(d), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ds, &hs, sizeof(hs), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        const unsigned g = (unsigned)std::min(d.ntiles, 2048);
        if (p == 3) {
            hipLaunchKernelGGL(k_test_tile_moments<3>, dim3(g), dim3(TILE), 0, st, dd, theta, logw);
            hipLaunchKernelGGL(k_test_moments_finish<3>, dim3(1), dim3(TILE), 0, st, dd, ds);
        } else if (p == 5) {
            hipLaunchKernelGGL(k_test_tile_moments<5>, dim3(g), dim3(TILE), 0, st, dd, theta, logw);
            hipLaunchKernelGGL(k_test_moments_finish<5>, dim3(1), dim3(TILE), 0, st, dd, ds);
        } else {
            hipLaunchKernelGGL(k_test_tile_moments<12>, dim3(g), dim3(TILE), 0, st, dd, theta, logw);
            hipLaunchKernelGGL(k_test_moments_finish<12>, dim3(1), dim3(TILE), 0, st, dd, ds);
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hs, ds, sizeof(hs), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(PF_EDEVICE, std::string("moments: ") + hipGetErrorString(e));
    if (hs.status != ST_OK) return fail((pf_status)hs.status, "every weight zero or covariance not factorable");
    for (uint32_t i = 0; i < p; ++i) {
        if (mean) mean[i] = hs.theta_bar[i];
        for (uint32_t j = 0; j < p; ++j) {
            if (cov) cov[i * p + j] = hs.C[i * p + j];
            if (chol) chol[i * p + j] = hs.L[i * p + j];
        }
    }
    if (ess) *ess = hs.ess;
    return PF_OK;
}

// The filter-based test entry points run on the context's own stream, which
// does not wait for the caller's streams: they first wait for the whole
// device, so the caller's buffers are ready (e.g. still being cleared on
// another stream) before the library writes or reads them.
extern "C" pf_status pf_test_get_ensemble(pf_filter* f, double* x, double* theta, double* logw)
{
    if (!f) return fail(PF_EINVAL, "NULL filter");
    pf_context* ctx = f->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    pf_status s = drain(f, f->next_seq - 1);
    if (s != PF_OK) return s;
    const unsigned g = (unsigned)((f->desc.n + 255) / 256);
    if (f->desc.prec == PREC_FP32)
        hipLaunchKernelGGL(k_test_get<float>, dim3(g), dim3(256), 0, ctx->stream, ctx->d_desc, ctx->d_state, f->slot, x,
                           theta, logw);
    else
        hipLaunchKernelGGL(k_test_get<double>, dim3(g), dim3(256), 0, ctx->stream, ctx->d_desc, ctx->d_state, f->slot, x,
                           theta, logw);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (logw) {
        // normalise on the host (test path only)
        std::vector<double> h(f->desc.n);
        HIP_TRY(hipMemcpy(h.data(), logw, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
        double mx = -INFINITY;
        for (double v : h) mx = std::max(mx, v);
        double sum = 0.0;
        for (double v : h) sum += v > -INFINITY ? std::exp(v - mx) : 0.0;
        const double lz = mx + std::log(sum);
        for (double& v : h) v = v > -INFINITY ? v - lz : -INFINITY;
        HIP_TRY(hipMemcpy(logw, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
    }
    return PF_OK;
}

extern "C" pf_status pf_test_set_ensemble(pf_filter* f, const double* x, const double* theta, const double* logw,
                                          const double* theta_bar, const double* L, uint64_t step, double t)
{
    if (!f || !x || !theta || !logw || !theta_bar || !L) return fail(PF_EINVAL, "NULL argument");
    pf_context* ctx = f->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    pf_status s = drain(f, f->next_seq - 1);
    if (s != PF_OK) return s;
    const unsigned g = (unsigned)((f->desc.n + 255) / 256);
    if (f->desc.prec == PREC_FP32)
        hipLaunchKernelGGL(k_test_set<float>, dim3(g), dim3(256), 0, ctx->stream, ctx->d_desc, ctx->d_state, f->slot, x,
                           theta, logw);
    else
        hipLaunchKernelGGL(k_test_set<double>, dim3(g), dim3(256), 0, ctx->stream, ctx->d_desc, ctx->d_state, f->slot, x,
                           theta, logw);
    HIP_TRY(hipGetLastError());
    FilterState st;
    HIP_TRY(hipMemcpyAsync(&st, ctx->d_state + f->slot, sizeof(st), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    const int p = f->desc.p;
    for (int i = 0; i < p; ++i) st.theta_bar[i] = theta_bar[i];
    for (int i = 0; i < p * p; ++i) st.L[i] = L[i];
    st.j = step;
    st.t = t;
    HIP_TRY(hipMemcpyAsync(ctx->d_state + f->slot, &st, sizeof(st), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    f->t_submitted = t;
    return PF_OK;
}

extern "C" pf_status pf_test_last_ancestors(pf_filter* f, int32_t* anc)
{
    if (!f || !anc) return fail(PF_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(f->ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    pf_status s = drain(f, f->next_seq - 1);
    if (s != PF_OK) return s;
    HIP_TRY(hipMemcpyAsync(anc, f->desc.anc, sizeof(int32_t) * f->desc.n, hipMemcpyDeviceToDevice, f->ctx->stream));
    HIP_TRY(hipStreamSynchronize(f->ctx->stream));
    return PF_OK;
}

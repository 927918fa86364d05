// Host-only stand-in for the part of the filter ABI (include/pf.h) that the
// serving loop uses: pf_create, pf_assimilate_batch, pf_query, pf_posterior,
// pf_destroy, pf_filter_bytes, pf_context_memory.  A batch's steps complete
// at a random time up to 2 ms after submission (in order per filter, out of
// order across batches, as with batches on several streams), so the
// server's admission, tick, completion and release bookkeeping runs on the
// CPU, under sanitizers, with no GPU.  main() opens N streams and submits
// every observation at once, without pacing, then drains and checks counts.
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include "pf.h"

using Clock = std::chrono::steady_clock;
struct pf_context { std::mutex mu; uint64_t used = 0, cap = 48ull << 30; std::mt19937_64 rng{1}; };
struct Tk { uint64_t seq; Clock::time_point done; };
struct pf_filter { pf_context* ctx; uint64_t next_seq = 1; std::deque<Tk> pending; std::map<uint64_t,int> done_status; uint64_t bytes; double t = -1e300; };

extern "C" {
uint64_t pf_filter_bytes(const pf_config* cfg) { return cfg ? (1ull << 20) * (1 + cfg->n_particles / 4096) : 0; }
pf_status pf_context_memory(pf_context* ctx, uint64_t* used, uint64_t* cap) { std::lock_guard<std::mutex> l(ctx->mu); *used = ctx->used; *cap = ctx->cap; return PF_OK; }
pf_status pf_create(pf_context* ctx, const pf_config* cfg, pf_filter** out) {
    std::lock_guard<std::mutex> l(ctx->mu);
    auto* f = new pf_filter(); f->ctx = ctx; f->bytes = pf_filter_bytes(cfg); ctx->used += f->bytes; *out = f; return PF_OK; }
static thread_local const char* last = "";
const char* pf_last_error(void) { return last; }
const char* pf_status_str(pf_status) { return ""; }
pf_status pf_assimilate_batch(pf_context* ctx, uint32_t n, pf_filter* const* fs, const double* t, const double* y, const double* s, uint64_t* tk) {
    std::lock_guard<std::mutex> l(ctx->mu);
    for (uint32_t i = 0; i < n; ++i) {
        for (uint32_t c = 0; c < i; ++c) if (fs[c] == fs[i]) return PF_EINVAL;
        if (fs[i]->pending.size() >= 64) return PF_EBUSY;
        if (!(t[i] > fs[i]->t)) return PF_EORDER;
    }
    // ticks complete out of order across batches (two streams), in order per filter
    const auto base = Clock::now() + std::chrono::microseconds(ctx->rng() % 2000);
    for (uint32_t i = 0; i < n; ++i) {
        pf_filter* f = fs[i];
        auto d = base;
        if (!f->pending.empty() && f->pending.back().done > d) d = f->pending.back().done + std::chrono::microseconds(1);
        f->pending.push_back({f->next_seq, d});
        f->t = t[i];
        tk[i] = f->next_seq++;
    }
    return PF_OK;
}
pf_status pf_query(pf_filter* f, uint64_t ticket) {
    if (ticket == 0 || ticket >= f->next_seq) return PF_EINVAL;
    const auto now = Clock::now();
    while (!f->pending.empty() && f->pending.front().seq <= ticket) {
        if (f->pending.front().done > now) return PF_EBUSY;
        f->done_status[f->pending.front().seq] = PF_OK;
        f->pending.pop_front();
    }
    auto it = f->done_status.find(ticket);
    if (it == f->done_status.end()) return PF_EINVAL;
    const int st = it->second; f->done_status.erase(it); return (pf_status)st;
}
pf_status pf_posterior(pf_filter* f, double* mean, double* cov, double* sm, double* ess, uint64_t* step) {
    while (!f->pending.empty()) { std::this_thread::sleep_until(f->pending.back().done); f->pending.clear(); }
    if (mean) std::memset(mean, 0, 8 * 3); if (cov) std::memset(cov, 0, 8 * 9); if (ess) *ess = 1; if (step) *step = f->next_seq - 1; return PF_OK; }
void pf_destroy(pf_filter* f) { { std::lock_guard<std::mutex> l(f->ctx->mu); f->ctx->used -= f->bytes; } delete f; }
}

int main(int argc, char** argv) {
    const int nstreams = argc > 1 ? atoi(argv[1]) : 500, T = 50;
    pf_context ctx;
    pf_server* s = nullptr;
    pf_server_config sc{sizeof(pf_server_config), 3, 4096, 0};
    if (pf_server_create(&ctx, &sc, &s) != PF_OK) return 1;
    uint32_t obs = 1; double x0[3] = {1, 0, 0}, pm[3] = {0, 0, 0}, ps[3] = {1, 1, 1}, fl[3] = {1e-6, 1e-6, 1e-6};
    pf_config cfg{}; cfg.struct_size = sizeof(pf_config); cfg.model = (pf_model)1; cfg.d = 3; cfg.p = 3; cfg.m = 1;
    cfg.obs_index = &obs; cfg.x0 = x0; cfg.prior_mean = pm; cfg.prior_sd = ps; cfg.state_floor = fl;
    std::vector<uint64_t> sid(nstreams);
    for (int k = 0; k < nstreams; ++k) { cfg.n_particles = 4096u << (k % 3); if (pf_server_open(s, &cfg, &sid[k]) != PF_OK) return 2; }
    for (int j = 0; j < T; ++j)
        for (int k = 0; k < nstreams; ++k) {
            const int Tk_ = (k % 10 < 7) ? T / 2 : T;
            if (j < Tk_) {
                double y = 1, sg = 0.1; uint64_t tk;
                if (pf_server_submit(s, sid[k], 1.0 + j, &y, &sg, &tk) != PF_OK) return 3;
                if (j == Tk_ - 1) pf_server_close(s, sid[k]);
            }
        }
    pf_server_drain(s);
    pf_server_report r{};
    pf_server_stats(s, &r);
    printf("ticks %lu completed %lu skipped %lu closed %lu\n", (unsigned long)r.ticks,
           (unsigned long)r.steps_completed, (unsigned long)r.steps_skipped, (unsigned long)r.streams_closed);
    pf_server_destroy(s);
    return 0;
}

// pf_server.cpp -- continuous-batching serving loop over the C ABI of
// include/pf.h: a scheduler thread admits streams by pool memory (first
// come, first served), launches ticks (one batched step over the oldest
// pending observation of every admitted stream that has one), keeps up to
// max_inflight ticks on the GPU, and records each step's latency from
// submission to observed completion.  It uses only the public filter API, so
// a served stream computes exactly what the same filter computes alone.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pf.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double fr = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1.0 - fr) + v[i + 1] * fr : v[i];
}

// deep copy of a pf_config with its arrays
struct OwnedConfig {
    pf_config cfg{};
    std::vector<uint32_t> obs;
    std::vector<double> mc, rf, x0, pm, ps, fl;

    explicit OwnedConfig(const pf_config& c) : cfg(c)
    {
        obs.assign(c.obs_index, c.obs_index + c.m);
        if (c.model_consts) mc.assign(c.model_consts, c.model_consts + c.n_model_consts);
        if (c.rates_fixed) rf.assign(c.rates_fixed, c.rates_fixed + c.n_rates_fixed);
        x0.assign(c.x0, c.x0 + c.d);
        pm.assign(c.prior_mean, c.prior_mean + c.p);
        ps.assign(c.prior_sd, c.prior_sd + c.p);
        fl.assign(c.state_floor, c.state_floor + c.d);
        cfg.obs_index = obs.data();
        cfg.model_consts = mc.empty() ? nullptr : mc.data();
        cfg.rates_fixed = rf.empty() ? nullptr : rf.data();
        cfg.x0 = x0.data();
        cfg.prior_mean = pm.data();
        cfg.prior_sd = ps.data();
        cfg.state_floor = fl.data();
    }
};

struct Obs {
    uint64_t ticket;
    double t;
    double y[4], sigma[4];
    Clock::time_point submitted;
};

struct InFlight {
    uint64_t ticket;      // server ticket
    uint64_t fticket;     // filter ticket
    Clock::time_point submitted;
};

struct Result {
    pf_status status;
    double latency_ms;
};

enum class SState { Queued, Active, Closing, Closed };

struct Stream {
    uint64_t id = 0;
    OwnedConfig conf;
    SState state = SState::Queued;
    bool close_requested = false;
    int readers = 0;                  // pf_server_posterior calls reading f outside the lock
    pf_filter* f = nullptr;
    uint64_t bytes = 0;
    uint64_t next_ticket = 1;
    double last_t = -INFINITY;
    std::deque<Obs> waiting;          // submitted, not yet launched
    std::deque<InFlight> inflight;    // launched, not yet observed complete
    uint64_t completed_upto = 0;      // tickets complete in order: all <= this are done
    std::map<uint64_t, Result> done;  // completed, not yet polled
    Clock::time_point opened;
    // posterior kept when the stream is released
    bool has_final = false;
    double fmean[12], fcov[144], fess = 0.0;
    uint64_t fstep = 0;

    explicit Stream(const pf_config& c) : conf(c) {}
};

}  // namespace

struct pf_server {
    pf_context* ctx = nullptr;
    uint32_t max_inflight = 3, max_batch = 4096;
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler
    std::condition_variable done_cv;  // wakes waiters on completions
    std::thread worker;
    bool stop = false;
    uint64_t next_id = 1;
    std::map<uint64_t, Stream*> streams;
    std::deque<uint64_t> admit_queue;
    std::map<uint64_t, Stream*> live;                   // admitted streams with waiting or in-flight steps
    // launched ticks: (stream id, server ticket) of each member
    std::deque<std::vector<std::pair<uint64_t, uint64_t>>> ticks_inflight;
    // stats
    uint64_t opened = 0, admitted = 0, closed = 0, ticks = 0, completed = 0, skipped = 0, psteps = 0;
    uint64_t batch_sum = 0;
    std::vector<double> latencies, admit_waits;
    bool any_submit = false;
    Clock::time_point first_submit, last_done;
    std::string worker_error;

    void loop();
    bool admit_locked();
    bool collect_locked();
    bool launch_locked();
    void release_locked(Stream* s);
};

void pf_server::release_locked(Stream* s)
{
    if (s->f) {
        s->has_final = pf_posterior(s->f, s->fmean, s->fcov, nullptr, &s->fess, &s->fstep) == PF_OK;
        pf_destroy(s->f);
    }
    s->f = nullptr;
    s->state = SState::Closed;
    closed++;
}

// admit queued streams in arrival order while the pool has room
bool pf_server::admit_locked()
{
    bool progress = false;
    while (!admit_queue.empty()) {
        Stream* s = streams[admit_queue.front()];
        if (s->close_requested && s->waiting.empty()) {   // closed before admission
            admit_queue.pop_front();
            s->state = SState::Closed;
            closed++;
            progress = true;
            continue;
        }
        pf_filter* f = nullptr;
        const pf_status st = pf_create(ctx, &s->conf.cfg, &f);
        if (st == PF_EADMIT) break;   // head of line waits for memory
        admit_queue.pop_front();
        progress = true;
        if (st != PF_OK) {
            // cannot run: fail its queued observations
            for (const Obs& o : s->waiting) s->done[o.ticket] = Result{st, 0.0};
            s->waiting.clear();
            s->state = SState::Closed;
            closed++;
            done_cv.notify_all();
            continue;
        }
        s->f = f;
        s->state = SState::Active;
        admitted++;
        admit_waits.push_back(ms_between(s->opened, Clock::now()));
        if (!s->waiting.empty() || s->close_requested) live[s->id] = s;
        done_cv.notify_all();   // a posterior call may wait for the admission
    }
    return progress;
}

// observe completed steps of in-flight ticks (in order per stream)
bool pf_server::collect_locked()
{
    bool progress = false;
    const auto now = Clock::now();
    for (auto it = live.begin(); it != live.end();) {
        Stream* s = it->second;
        while (!s->inflight.empty()) {
            InFlight& h = s->inflight.front();
            const pf_status st = pf_query(s->f, h.fticket);
            if (st == PF_EBUSY) break;
            const double lat = ms_between(h.submitted, now);
            s->done[h.ticket] = Result{st, lat};
            s->completed_upto = h.ticket;
            latencies.push_back(lat);
            if (st == PF_OK) {
                completed++;
                psteps += s->conf.cfg.n_particles;
            } else {
                skipped++;
            }
            last_done = now;
            s->inflight.pop_front();
            progress = true;
        }
        if (s->waiting.empty() && s->inflight.empty()) {
            if (s->close_requested && s->readers > 0) {
                ++it;   // released once the posterior read ends
                continue;
            }
            if (s->close_requested) release_locked(s);
            it = live.erase(it);
            progress = true;
        } else {
            ++it;
        }
    }
    // retire ticks whose members have all completed
    while (!ticks_inflight.empty()) {
        bool all = true;
        for (const auto& m : ticks_inflight.front())
            if (streams[m.first]->completed_upto < m.second) { all = false; break; }
        if (!all) break;
        ticks_inflight.pop_front();
        progress = true;
    }
    if (progress) done_cv.notify_all();
    return progress;
}

// one tick: the oldest waiting observation of each admitted stream
bool pf_server::launch_locked()
{
    if (ticks_inflight.size() >= max_inflight) return false;
    std::vector<Stream*> members;
    for (auto& kv : live) {
        Stream* s = kv.second;
        // a stream whose posterior is being read is not touched until the read ends
        if (!s->waiting.empty() && s->inflight.size() < 60 && s->readers == 0) members.push_back(s);
        if (members.size() >= max_batch) break;
    }
    if (members.empty()) return false;
    const size_t n = members.size();
    std::vector<pf_filter*> fs(n);
    std::vector<double> t(n), y(4 * n), sg(4 * n);
    std::vector<uint64_t> tk(n);
    for (size_t i = 0; i < n; ++i) {
        const Obs& o = members[i]->waiting.front();
        fs[i] = members[i]->f;
        t[i] = o.t;
        for (int c = 0; c < 4; ++c) {
            y[4 * i + c] = o.y[c];
            sg[4 * i + c] = o.sigma[c];
        }
    }
    const pf_status st = pf_assimilate_batch(ctx, (uint32_t)n, fs.data(), t.data(), y.data(), sg.data(), tk.data());
    if (st != PF_OK) {
        // observations were validated on submission, so this is a device
        // error: fail this tick's observations and keep serving
        worker_error = pf_last_error();
        for (Stream* s : members) {
            const Obs o = s->waiting.front();
            s->waiting.pop_front();
            s->done[o.ticket] = Result{st, 0.0};
            // with earlier steps still in flight, completed_upto advances when
            // they complete (the failed step belongs to no tick)
            if (s->inflight.empty()) s->completed_upto = o.ticket;
            skipped++;
        }
        done_cv.notify_all();
        return true;
    }
    std::vector<std::pair<uint64_t, uint64_t>> ids(n);
    for (size_t i = 0; i < n; ++i) {
        Stream* s = members[i];
        const Obs o = s->waiting.front();
        s->waiting.pop_front();
        s->inflight.push_back(InFlight{o.ticket, tk[i], o.submitted});
        ids[i] = {s->id, o.ticket};
    }
    ticks_inflight.push_back(std::move(ids));
    ticks++;
    batch_sum += n;
    return true;
}

void pf_server::loop()
{
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
        bool progress = admit_locked();
        progress |= collect_locked();
        progress |= launch_locked();
        if (!progress) {
            // work on the GPU: poll again shortly; otherwise sleep until woken
            const bool busy = !ticks_inflight.empty();
            cv.wait_for(lk, busy ? std::chrono::microseconds(20) : std::chrono::milliseconds(5));
        }
    }
}

extern "C" pf_status pf_server_create(pf_context* ctx, const pf_server_config* cfg, pf_server** out)
{
    if (!ctx || !out) return PF_EINVAL;
    if (cfg && cfg->struct_size != sizeof(pf_server_config)) return PF_EINVAL;
    auto* s = new pf_server();
    s->ctx = ctx;
    if (cfg && cfg->max_inflight) s->max_inflight = cfg->max_inflight;
    if (cfg && cfg->max_batch) s->max_batch = std::min<uint32_t>(cfg->max_batch, 4096);
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return PF_OK;
}

extern "C" pf_status pf_server_open(pf_server* s, const pf_config* cfg, uint64_t* stream)
{
    if (!s || !cfg || !stream) return PF_EINVAL;
    // served steps go through batched submissions, whose rows hold 4 observations
    if (cfg->m > 4) return PF_EINVAL;
    const uint64_t need = pf_filter_bytes(cfg);
    if (need == 0) return PF_EINVAL;
    uint64_t used = 0, cap = 0;
    pf_context_memory(s->ctx, &used, &cap);
    if (need > cap) return PF_ENOMEM;
    auto* st = new Stream(*cfg);
    std::lock_guard<std::mutex> lk(s->mu);
    st->id = s->next_id++;
    st->bytes = need;
    st->opened = Clock::now();
    s->streams[st->id] = st;
    s->admit_queue.push_back(st->id);
    s->opened++;
    *stream = st->id;
    s->cv.notify_one();
    return PF_OK;
}

extern "C" pf_status pf_server_submit(pf_server* s, uint64_t stream, double t_obs, const double* y,
                                      const double* sigma, uint64_t* ticket)
{
    if (!s || !y || !sigma) return PF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->streams.find(stream);
    if (it == s->streams.end()) return PF_EINVAL;
    Stream* st = it->second;
    if (st->close_requested || st->state == SState::Closed) return PF_EINVAL;
    if (!std::isfinite(t_obs) || !(t_obs > st->last_t)) return PF_EORDER;
    for (uint32_t c = 0; c < st->conf.cfg.m; ++c)
        if (!std::isfinite(y[c]) || !std::isfinite(sigma[c]) || !(sigma[c] > 0.0)) return PF_EINVAL;
    Obs o{};
    o.ticket = st->next_ticket++;
    o.t = t_obs;
    for (uint32_t c = 0; c < st->conf.cfg.m && c < 4; ++c) {
        o.y[c] = y[c];
        o.sigma[c] = sigma[c];
    }
    o.submitted = Clock::now();
    if (!s->any_submit) {
        s->any_submit = true;
        s->first_submit = o.submitted;
    }
    st->last_t = t_obs;
    st->waiting.push_back(o);
    if (st->state == SState::Active) s->live[st->id] = st;
    if (ticket) *ticket = o.ticket;
    s->cv.notify_one();
    return PF_OK;
}

extern "C" pf_status pf_server_poll(pf_server* s, uint64_t stream, uint64_t ticket, double* latency_ms)
{
    if (!s) return PF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->streams.find(stream);
    if (it == s->streams.end()) return PF_EINVAL;
    Stream* st = it->second;
    auto d = st->done.find(ticket);
    if (d == st->done.end()) return ticket < st->next_ticket ? PF_EBUSY : PF_EINVAL;
    const Result r = d->second;
    st->done.erase(d);
    if (latency_ms) *latency_ms = r.latency_ms;
    return r.status;
}

extern "C" pf_status pf_server_posterior(pf_server* s, uint64_t stream, double* mean, double* cov, double* ess,
                                         uint64_t* step)
{
    if (!s) return PF_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->streams.find(stream);
    if (it == s->streams.end()) return PF_EINVAL;
    Stream* st = it->second;
    s->cv.notify_one();
    s->done_cv.wait(lk, [&] {
        return st->state == SState::Closed || (st->state != SState::Queued && st->waiting.empty() && st->inflight.empty());
    });
    if (!st->f) {
        // closed: the summary kept at release (none if it was never admitted)
        if (!st->has_final) return PF_EINVAL;
        const uint32_t p = st->conf.cfg.p;
        if (mean) std::memcpy(mean, st->fmean, sizeof(double) * p);
        if (cov) std::memcpy(cov, st->fcov, sizeof(double) * p * p);
        if (ess) *ess = st->fess;
        if (step) *step = st->fstep;
        return PF_OK;
    }
    // read outside the lock (pf_posterior waits for the device): while
    // readers > 0 the scheduler launches nothing for this stream and does not
    // release it, so the filter has one user at a time
    st->readers++;
    pf_filter* f = st->f;
    lk.unlock();
    const pf_status r = pf_posterior(f, mean, cov, nullptr, ess, step);
    lk.lock();
    st->readers--;
    s->cv.notify_one();
    return r;
}

extern "C" pf_status pf_server_close(pf_server* s, uint64_t stream)
{
    if (!s) return PF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->streams.find(stream);
    if (it == s->streams.end()) return PF_EINVAL;
    Stream* st = it->second;
    st->close_requested = true;
    if (st->state == SState::Active) s->live[st->id] = st;
    s->cv.notify_one();
    return PF_OK;
}

extern "C" pf_status pf_server_drain(pf_server* s)
{
    if (!s) return PF_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.notify_one();
    s->done_cv.wait(lk, [&] {
        for (auto& kv : s->streams) {
            const Stream* st = kv.second;
            if (!st->waiting.empty() || !st->inflight.empty()) return false;
            if (st->close_requested && st->state != SState::Closed) return false;
        }
        return true;
    });
    return PF_OK;
}

extern "C" pf_status pf_server_stats(pf_server* s, pf_server_report* out)
{
    if (!s || !out) return PF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->streams_opened = s->opened;
    out->streams_admitted = s->admitted;
    out->streams_closed = s->closed;
    out->ticks = s->ticks;
    out->steps_completed = s->completed;
    out->steps_skipped = s->skipped;
    out->particle_steps = s->psteps;
    out->latency_p50_ms = percentile(s->latencies, 0.50);
    out->latency_p99_ms = percentile(s->latencies, 0.99);
    out->latency_max_ms = s->latencies.empty() ? 0.0 : *std::max_element(s->latencies.begin(), s->latencies.end());
    out->admit_wait_p50_ms = percentile(s->admit_waits, 0.50);
    out->admit_wait_p99_ms = percentile(s->admit_waits, 0.99);
    out->mean_batch = s->ticks ? (double)s->batch_sum / (double)s->ticks : 0.0;
    out->busy_s = s->any_submit ? ms_between(s->first_submit, s->last_done) / 1e3 : 0.0;
    return PF_OK;
}

extern "C" void pf_server_destroy(pf_server* s)
{
    if (!s) return;
    pf_server_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_one();
    }
    s->worker.join();
    for (auto& kv : s->streams) {
        if (kv.second->f) pf_destroy(kv.second->f);
        delete kv.second;
    }
    delete s;
}

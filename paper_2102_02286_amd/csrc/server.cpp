// server.cpp -- continuous-batching search server over a resident index.
//
// The index stays in HBM.  The caller's device pool is divided into slots;
// each slot is a search plan (its own stream and captured graph) for up to
// slot_spectra spectra.  A scheduler thread admits queued requests in arrival
// order: whenever a slot is free it packs as many waiting requests as fit the
// slot's capacity into one run, so requests that arrive while other runs are
// on the GPU are admitted as slots free up, and runs on different slots overlap
// on the device.  This is the GPU analogue of the paper's producer/consumer
// pipeline with recycled buffers (Superstep 3, Buffering): the slots are the
// buffers, the request queue is the forward queue.  Results are per request
// and identical to searching the request alone (every spectrum's result depends
// only on that spectrum).
#include "batch.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace ps;
using Clock = std::chrono::steady_clock;

extern "C" {
int ps_plan_bytes(const ps_index* ix, uint64_t n_cap, uint64_t nnz_cap, const ps_search_params* params,
                  uint64_t* bytes);
int ps_plan_create(ps_index* ix, const ps_device* work, uint64_t n_cap, uint64_t nnz_cap,
                   const ps_search_params* params, ps_plan** out);
int ps_plan_run(ps_plan* plan, const ps_spectra* spectra);
int ps_plan_results(ps_plan* plan, ps_hit* hits, ps_stat* stats, int32_t* hist);
void ps_plan_free(ps_plan* plan);
}

namespace {

struct Request {
    uint64_t ticket = 0;
    std::vector<uint64_t> off;
    std::vector<float> mz, in;
    std::vector<double> prec;
    std::vector<int8_t> z;
    Clock::time_point t_submit, t_admit, t_done;
    bool done = false;
    int rc = PS_OK;
    std::vector<ps_hit> hits;
    std::vector<ps_stat> stats;
    std::vector<int32_t> hist;
    uint64_t n() const { return off.size() - 1; }
    uint64_t nnz() const { return off.back(); }
};

struct Slot {
    ps_plan* plan = nullptr;
    bool busy = false;
    std::vector<Request*> reqs;   // requests packed into the current run
    // staging for the packed run
    std::vector<uint64_t> off;
    std::vector<float> mz, in;
    std::vector<double> prec;
    std::vector<int8_t> z;
};

}  // namespace

struct ps_server {
    ps_index* ix = nullptr;
    ps_search_params prm{};
    uint64_t slot_n = 0, slot_nnz = 0, slot_bytes = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, Request*> all;
    uint64_t next_ticket = 1;
    uint64_t max_pending = 0;
    bool stop = false;
    std::thread sched;
    // statistics
    std::vector<double> latencies_ms;
    uint64_t completed = 0, spectra_done = 0, runs = 0, refused = 0, max_depth = 0;
    Clock::time_point t_first{}, t_last{};
    bool have_first = false;
    std::atomic<int> error{PS_OK};
};

static void pack_and_run(ps_server* S, Slot& sl) {
    // caller holds S->mu; moves requests from pending into the slot
    sl.reqs.clear();
    uint64_t n = 0, nnz = 0;
    while (!S->pending.empty()) {
        Request* r = S->pending.front();
        if (!sl.reqs.empty() && (n + r->n() > S->slot_n || nnz + r->nnz() > S->slot_nnz)) break;
        S->pending.pop_front();
        sl.reqs.push_back(r);
        n += r->n();
        nnz += r->nnz();
    }
    sl.off.assign(1, 0);
    sl.mz.clear(); sl.in.clear(); sl.prec.clear(); sl.z.clear();
    const auto now = Clock::now();
    for (Request* r : sl.reqs) {
        r->t_admit = now;
        const uint64_t base = sl.off.back();
        for (uint64_t i = 1; i < r->off.size(); ++i) sl.off.push_back(base + r->off[i]);
        sl.mz.insert(sl.mz.end(), r->mz.begin(), r->mz.end());
        sl.in.insert(sl.in.end(), r->in.begin(), r->in.end());
        sl.prec.insert(sl.prec.end(), r->prec.begin(), r->prec.end());
        sl.z.insert(sl.z.end(), r->z.begin(), r->z.end());
    }
    ps_spectra sp;
    sp.n = n;
    sp.peak_off = sl.off.data();
    sp.mz = sl.mz.data();
    sp.intensity = sl.in.data();
    sp.precursor_mz = sl.prec.data();
    sp.charge = sl.z.data();
    const int rc = ps_plan_run(sl.plan, &sp);
    if (rc != PS_OK) {
        for (Request* r : sl.reqs) { r->rc = rc; r->done = true; r->t_done = Clock::now(); }
        sl.reqs.clear();
        S->cv_done.notify_all();
        return;
    }
    sl.busy = true;
    ++S->runs;
}

// Copy a finished slot's results back to its requests.
static void complete(ps_server* S, Slot& sl) {
    uint64_t n = 0;
    for (Request* r : sl.reqs) n += r->n();
    const uint32_t k = S->prm.top_k;
    std::vector<ps_hit> hits(n * k);
    std::vector<ps_stat> stats(n);
    std::vector<int32_t> hist(S->prm.want_hist ? n * (uint64_t)kHistBins : 0);
    const int rc = ps_plan_results(sl.plan, hits.data(), stats.data(), S->prm.want_hist ? hist.data() : nullptr);
    const auto now = Clock::now();
    uint64_t at = 0;
    for (Request* r : sl.reqs) {
        const uint64_t m = r->n();
        r->hits.assign(hits.begin() + at * k, hits.begin() + (at + m) * k);
        r->stats.assign(stats.begin() + at, stats.begin() + at + m);
        if (S->prm.want_hist)
            r->hist.assign(hist.begin() + at * kHistBins, hist.begin() + (at + m) * kHistBins);
        at += m;
        r->rc = rc == PS_EOVERFLOW ? PS_OK : rc;
        r->done = true;
        r->t_done = now;
        S->latencies_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
        ++S->completed;
        S->spectra_done += m;
    }
    S->t_last = now;
    sl.reqs.clear();
    sl.busy = false;
}

extern "C" int ps_plan_event_query(ps_plan* plan);   // plan.cpp

static void scheduler(ps_server* S) {
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        bool progressed = false;
        // completions
        for (Slot& sl : S->slots) {
            if (!sl.busy) continue;
            const int q = ps_plan_event_query(sl.plan);
            if (q == 0) continue;                 // still running
            complete(S, sl);
            progressed = true;
        }
        if (progressed) S->cv_done.notify_all();
        // admissions: fill every free slot from the queue
        for (Slot& sl : S->slots) {
            if (S->pending.empty()) break;
            if (sl.busy) continue;
            pack_and_run(S, sl);
            progressed = true;
        }
        bool any_busy = false;
        for (Slot& sl : S->slots) any_busy |= sl.busy;
        if (S->stop && S->pending.empty() && !any_busy) break;
        if (!progressed) {
            if (any_busy) {
                // poll device completion without holding the lock for long
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            }
        }
    }
}

extern "C" int ps_server_create(ps_index* ix, const ps_device* pool, const ps_search_params* params,
                                uint64_t slot_spectra, uint64_t slot_peaks, uint32_t max_slots,
                                uint64_t max_pending, ps_server** out) {
    if (!out) return fail(PS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ix || !pool || !params) return fail(PS_EINVAL, "NULL argument");
    if (slot_spectra == 0 || slot_peaks == 0 || max_slots == 0)
        return fail(PS_EINVAL, "slot sizes and max_slots must be positive");
    if (params->schedule != PS_SCHED_PERSISTENT) return fail(PS_EINVAL, "the server runs the persistent schedule");
    uint64_t per = 0;
    int rc = ps_plan_bytes(ix, slot_spectra, slot_peaks, params, &per);
    if (rc != PS_OK) return rc;
    per = (per + 255) & ~255ull;
    const uint64_t fit = pool->bytes / per;
    if (fit == 0)
        return fail(PS_ENOMEM, "pool of %llu bytes holds no slot of %llu bytes", (unsigned long long)pool->bytes,
                    (unsigned long long)per);
    ps_server* S = new (std::nothrow) ps_server();
    if (!S) return fail(PS_ENOMEM, "out of host memory");
    S->ix = ix;
    S->prm = *params;
    S->slot_n = slot_spectra;
    S->slot_nnz = slot_peaks;
    S->slot_bytes = per;
    S->max_pending = max_pending ? max_pending : (1ull << 20);
    const uint64_t ns = std::min<uint64_t>(fit, max_slots);
    S->slots.resize(ns);
    for (uint64_t i = 0; i < ns; ++i) {
        ps_device d;
        d.base = (char*)pool->base + i * per;
        d.bytes = per;
        d.stream = nullptr;                     // each slot gets its own stream
        rc = ps_plan_create(ix, &d, slot_spectra, slot_peaks, params, &S->slots[i].plan);
        if (rc != PS_OK) {
            for (auto& sl : S->slots) if (sl.plan) ps_plan_free(sl.plan);
            delete S;
            return rc;
        }
    }
    S->sched = std::thread(scheduler, S);
    *out = S;
    return PS_OK;
}

extern "C" int ps_server_submit(ps_server* S, const ps_spectra* sp, uint64_t* ticket) {
    if (!S || !sp || !ticket) return fail(PS_EINVAL, "NULL argument");
    KParams kp;
    Schedule sc = S->ix->sched;
    int rc = make_kparams(S->ix, &S->prm, &kp, &sc);
    if (rc != PS_OK) return rc;
    rc = validate_host_spectra(sp, kp);
    if (rc != PS_OK) return rc;
    const uint64_t n = sp->n, nnz = n ? sp->peak_off[n] : 0;
    if (n > S->slot_n || nnz > S->slot_nnz)
        return fail(PS_EINVAL, "request of %llu spectra / %llu peaks exceeds a slot (%llu / %llu)",
                    (unsigned long long)n, (unsigned long long)nnz, (unsigned long long)S->slot_n,
                    (unsigned long long)S->slot_nnz);
    Request* r = new (std::nothrow) Request();
    if (!r) return fail(PS_ENOMEM, "out of host memory");
    r->off.assign(sp->peak_off, sp->peak_off + n + 1);
    if (nnz) { r->mz.assign(sp->mz, sp->mz + nnz); r->in.assign(sp->intensity, sp->intensity + nnz); }
    r->prec.assign(sp->precursor_mz, sp->precursor_mz + n);
    r->z.assign(sp->charge, sp->charge + n);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (S->pending.size() >= S->max_pending) {
            ++S->refused;
            delete r;
            return fail(PS_EAGAIN, "request queue is full (%llu waiting)", (unsigned long long)S->pending.size());
        }
        r->ticket = S->next_ticket++;
        S->pending.push_back(r);
        S->all[r->ticket] = r;
        S->max_depth = std::max<uint64_t>(S->max_depth, S->pending.size());
        if (!S->have_first) { S->t_first = r->t_submit; S->have_first = true; }
    }
    S->cv_work.notify_one();
    *ticket = r->ticket;
    return PS_OK;
}

extern "C" int ps_server_wait(ps_server* S, uint64_t ticket, ps_hit* hits, ps_stat* stats, int32_t* hist,
                              double* latency_ms) {
    if (!S) return fail(PS_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(PS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second;
    S->cv_done.wait(lk, [&] { return r->done; });
    S->all.erase(it);
    lk.unlock();
    const int rc = r->rc;
    if (rc == PS_OK) {
        if (hits) memcpy(hits, r->hits.data(), r->hits.size() * sizeof(ps_hit));
        if (stats) memcpy(stats, r->stats.data(), r->stats.size() * sizeof(ps_stat));
        if (hist && S->prm.want_hist) memcpy(hist, r->hist.data(), r->hist.size() * sizeof(int32_t));
    }
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    delete r;
    return rc == PS_OK ? PS_OK : fail(rc, "request failed on the device");
}

extern "C" int ps_server_stats(ps_server* S, ps_serve_stats* out) {
    if (!S || !out) return fail(PS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    memset(out, 0, sizeof *out);
    out->completed = S->completed;
    out->spectra = S->spectra_done;
    out->runs = S->runs;
    out->refused = S->refused;
    out->max_queue = S->max_depth;
    out->slots = (uint32_t)S->slots.size();
    out->slot_bytes = S->slot_bytes;
    std::vector<double> v = S->latencies_ms;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const double pos = p * (double)(v.size() - 1);
            const size_t i = (size_t)pos;
            const double f = pos - (double)i;
            return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = v.back();
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_ms = sum / (double)v.size();
    }
    if (S->have_first && S->completed)
        out->elapsed_s = std::chrono::duration<double>(S->t_last - S->t_first).count();
    return PS_OK;
}

extern "C" int ps_server_reset_stats(ps_server* S) {
    if (!S) return fail(PS_EINVAL, "NULL server");
    std::lock_guard<std::mutex> g(S->mu);
    S->latencies_ms.clear();
    S->completed = S->spectra_done = S->runs = S->refused = S->max_depth = 0;
    S->have_first = false;
    return PS_OK;
}

extern "C" void ps_server_free(ps_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->sched.joinable()) S->sched.join();
    for (auto& sl : S->slots) if (sl.plan) ps_plan_free(sl.plan);
    for (auto& kv : S->all) delete kv.second;
    delete S;
}

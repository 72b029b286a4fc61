// server.cpp -- continuous-batching search server over a resident index.
//
// The index stays in HBM.  The caller's device pool is an arena: every run of
// the server reserves exactly the workspace its batch needs (inputs, entries,
// histograms, partial top-k lists, results) from it with a first-fit allocator
// and returns it when the run completes.  A scheduler thread admits queued
// requests in arrival order: whenever a stream is free it packs waiting
// requests into one run up to the packing target, reserves the run's bytes and
// enqueues the whole search on that stream, so requests that arrive while
// others are on the GPU are admitted as streams and memory free up, and runs on
// different streams overlap on the device.  A request that does not fit the
// free memory waits at the head of the queue (it is never skipped); a
// submission is refused with PS_EAGAIN while the bytes of queued and running
// requests would pass the server's limit.  This is the GPU analogue of the
// paper's producer/consumer pipeline with recycled buffers (Superstep 3,
// Buffering) and of the memory guard of Supplementary Algorithm 5, which stops
// taking in data while the memory in use is above a threshold.  Results are
// per request and identical to searching the request alone (every spectrum's
// result depends only on that spectrum).
#include "batch.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace ps;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    uint64_t ticket = 0;
    uint64_t need = 0;                 // device bytes of this request searched alone
    std::vector<uint64_t> off;
    std::vector<float> mz, in;
    std::vector<double> prec;
    std::vector<int8_t> z;
    Clock::time_point t_submit, t_admit, t_done;
    bool done = false;
    bool claimed = false;              // a waiter has taken the ticket
    int rc = PS_OK;
    std::vector<ps_hit> hits;
    std::vector<ps_stat> stats;
    std::vector<int32_t> hist;
    uint64_t n() const { return off.size() - 1; }
    uint64_t nnz() const { return off.back(); }
};

// First-fit allocator over [0, size) in 256-byte units; adjacent free ranges
// are merged on release.
class Arena {
public:
    explicit Arena(uint64_t size) : size_(size & ~255ull) { if (size_) free_[0] = size_; }
    bool alloc(uint64_t bytes, uint64_t* at) {
        bytes = (bytes + 255) & ~255ull;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *at = it->first;
            const uint64_t rest = it->second - bytes, next = it->first + bytes;
            free_.erase(it);
            if (rest) free_[next] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(uint64_t at, uint64_t bytes) {
        bytes = (bytes + 255) & ~255ull;
        if (bytes == 0) bytes = 256;
        used_ -= bytes;
        auto it = free_.emplace(at, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
        }
    }
    uint64_t size() const { return size_; }
    uint64_t peak() const { return peak_; }
    void reset_peak() { peak_ = used_; }

private:
    uint64_t size_, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

// One stream and what a run on it needs on the host side.
struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Request*> reqs;        // requests packed into the current run
    uint64_t off = 0, bytes = 0;       // its arena range
    uint64_t n = 0;
    // pinned staging, grown on demand
    char* h_in = nullptr;  uint64_t h_in_cap = 0;
    char* h_out = nullptr; uint64_t h_out_cap = 0;
    BatchHdr* h_hdr = nullptr;
};

}  // namespace

struct ps_server {
    ps_index* ix = nullptr;
    ps_search_params prm{};
    KParams kp{};
    Schedule sc{};
    char* pool = nullptr;
    uint64_t run_n = 0, run_nnz = 0, limit = 0;
    Arena arena{0};
    std::vector<Lane> lanes;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, Request*> all;
    uint64_t next_ticket = 1;
    uint64_t committed = 0;            // device bytes of queued and running requests
    bool stop = false;
    std::thread sched;
    // statistics
    std::vector<double> latencies_ms;
    uint64_t completed = 0, spectra_done = 0, runs = 0, refused = 0, max_depth = 0;
    Clock::time_point t_first{}, t_last{};
    bool have_first = false;
};

// Device bytes of one search of n spectra and nnz peaks in the server's settings.
static uint64_t run_bytes(const ps_server* S, uint64_t n, uint64_t nnz) {
    const uint64_t items = max_items_for(S->ix, n, S->kp, S->sc, S->prm.schedule);
    return layout_work(n, nnz, S->kp, true, items, nullptr, nullptr, nullptr, 0);
}

static hipError_t grow_pinned(char** p, uint64_t* cap, uint64_t need) {
    if (need <= *cap) return hipSuccess;
    uint64_t c = std::max<uint64_t>(need, 1ull << 20);
    c = 1ull << (64 - __builtin_clzll(c - 1));      // next power of two
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipHostMalloc((void**)p, c, hipHostMallocDefault);
    if (e == hipSuccess) *cap = c;
    return e;
}

static uint64_t out_bytes(const ps_server* S, uint64_t n) {
    return n * (uint64_t)S->prm.top_k * sizeof(ps_hit) + n * sizeof(ps_stat) +
           (S->prm.want_hist ? n * (uint64_t)kHistBins * 4 : 0);
}

// Stage the lane's requests, enqueue the whole search on its stream and the
// copies of the results back.  Called without the server lock.
static int enqueue_run(ps_server* S, Lane& L, uint64_t nnz) {
    const uint64_t n = L.n;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    const uint64_t o_mz = (n + 1) * 8, o_in = o_mz + nnz * 4, o_pr = o_in + nnz * 4, o_z = o_pr + n * 8;
    chk(grow_pinned(&L.h_in, &L.h_in_cap, o_z + n));
    chk(grow_pinned(&L.h_out, &L.h_out_cap, out_bytes(S, n)));
    if (e != hipSuccess) return fail(PS_EDEVICE, "server staging: %s", hipGetErrorString(e));
    uint64_t* off = (uint64_t*)L.h_in;
    off[0] = 0;
    uint64_t at = 0, pk = 0;
    for (Request* r : L.reqs) {
        for (uint64_t i = 1; i < r->off.size(); ++i) off[at + i] = pk + r->off[i];
        if (r->nnz()) {
            memcpy(L.h_in + o_mz + pk * 4, r->mz.data(), r->nnz() * 4);
            memcpy(L.h_in + o_in + pk * 4, r->in.data(), r->nnz() * 4);
        }
        memcpy(L.h_in + o_pr + at * 8, r->prec.data(), r->n() * 8);
        memcpy(L.h_in + o_z + at, r->z.data(), r->n());
        at += r->n();
        pk += r->nnz();
    }
    Work w;
    DevSpectra dsp;
    const uint64_t items = max_items_for(S->ix, n, S->kp, S->sc, S->prm.schedule);
    layout_work(n, nnz, S->kp, true, items, S->pool + L.off, &w, &dsp, 0);
    dsp.hdr = w.hdr;
    L.h_hdr->n = n;
    L.h_hdr->nnz = nnz;
    hipStream_t st = L.stream;
    chk(hipMemcpyAsync(w.hdr, L.h_hdr, sizeof(BatchHdr), hipMemcpyHostToDevice, st));
    chk(hipMemcpyAsync((void*)dsp.peak_off, L.h_in, (n + 1) * 8, hipMemcpyHostToDevice, st));
    if (nnz) {
        chk(hipMemcpyAsync((void*)dsp.mz, L.h_in + o_mz, nnz * 4, hipMemcpyHostToDevice, st));
        chk(hipMemcpyAsync((void*)dsp.inten, L.h_in + o_in, nnz * 4, hipMemcpyHostToDevice, st));
    }
    chk(hipMemcpyAsync((void*)dsp.prec, L.h_in + o_pr, n * 8, hipMemcpyHostToDevice, st));
    chk(hipMemcpyAsync((void*)dsp.charge, L.h_in + o_z, n, hipMemcpyHostToDevice, st));
    chk(enqueue_kernels(S->ix, dsp, S->kp, S->sc, S->prm.schedule, w, false, st, nullptr, nullptr));
    const uint64_t hb = n * (uint64_t)S->prm.top_k * sizeof(ps_hit), sb = n * sizeof(ps_stat);
    chk(hipMemcpyAsync(L.h_out, w.hits, hb, hipMemcpyDeviceToHost, st));
    chk(hipMemcpyAsync(L.h_out + hb, w.stats, sb, hipMemcpyDeviceToHost, st));
    if (S->prm.want_hist) chk(hipMemcpyAsync(L.h_out + hb + sb, w.hist, n * (uint64_t)kHistBins * 4,
                                             hipMemcpyDeviceToHost, st));
    chk(hipEventRecord(L.done, st));
    if (e != hipSuccess) return fail(PS_EDEVICE, "server run: %s", hipGetErrorString(e));
    return PS_OK;
}

// Copy a finished run's results back to its requests; caller holds the lock.
static void complete(ps_server* S, Lane& L, int rc) {
    const uint32_t k = S->prm.top_k;
    const ps_hit* hits = (const ps_hit*)L.h_out;
    const ps_stat* stats = (const ps_stat*)(L.h_out + L.n * k * sizeof(ps_hit));
    const int32_t* hist = (const int32_t*)(L.h_out + L.n * k * sizeof(ps_hit) + L.n * sizeof(ps_stat));
    const auto now = Clock::now();
    uint64_t at = 0;
    for (Request* r : L.reqs) {
        const uint64_t m = r->n();
        if (rc == PS_OK) {
            r->hits.assign(hits + at * k, hits + (at + m) * k);
            r->stats.assign(stats + at, stats + at + m);
            if (S->prm.want_hist) r->hist.assign(hist + at * kHistBins, hist + (at + m) * kHistBins);
        }
        at += m;
        r->rc = rc;
        r->done = true;
        r->t_done = now;
        S->committed -= r->need;
        if (rc == PS_OK) {
            S->latencies_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
            ++S->completed;
            S->spectra_done += m;
        }
    }
    S->t_last = now;
    S->arena.release(L.off, L.bytes);
    L.reqs.clear();
    L.busy = false;
}

// Take requests from the head of the queue for one run: as many as fit the
// packing target (at least one), and within that as many as fit the free
// memory.  Returns false when even the head request does not fit now.
static bool admit(ps_server* S, Lane& L, uint64_t* nnz_out) {
    uint64_t n = 0, nnz = 0;
    size_t take = 0;
    for (Request* r : S->pending) {
        if (take && (n + r->n() > S->run_n || nnz + r->nnz() > S->run_nnz)) break;
        n += r->n();
        nnz += r->nnz();
        ++take;
    }
    while (take) {
        const uint64_t bytes = run_bytes(S, n, nnz);
        uint64_t at = 0;
        if (S->arena.alloc(bytes, &at)) {
            L.off = at;
            L.bytes = bytes;
            break;
        }
        --take;                               // fewer requests, smaller run
        Request* r = S->pending[take];
        n -= r->n();
        nnz -= r->nnz();
    }
    if (!take) return false;
    const auto now = Clock::now();
    L.reqs.assign(S->pending.begin(), S->pending.begin() + take);
    S->pending.erase(S->pending.begin(), S->pending.begin() + take);
    for (Request* r : L.reqs) r->t_admit = now;
    L.n = n;
    L.busy = true;
    *nnz_out = nnz;
    return true;
}

static void scheduler(ps_server* S) {
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        bool progressed = false;
        for (Lane& L : S->lanes) {              // completions
            if (!L.busy || L.reqs.empty()) continue;
            const hipError_t q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) continue;
            complete(S, L, q == hipSuccess ? PS_OK : PS_EDEVICE);
            progressed = true;
        }
        if (progressed) S->cv_done.notify_all();
        for (Lane& L : S->lanes) {              // admissions
            if (S->pending.empty()) break;
            if (L.busy) continue;
            uint64_t nnz = 0;
            if (!admit(S, L, &nnz)) break;      // the head waits for memory
            ++S->runs;
            progressed = true;
            lk.unlock();                        // staging and launches need no lock
            const int rc = enqueue_run(S, L, nnz);
            // a run that failed part-way may have work queued on its range:
            // it must end before complete() returns the range to the arena
            if (rc != PS_OK) (void)hipStreamSynchronize(L.stream);
            lk.lock();
            if (rc != PS_OK) { complete(S, L, rc); S->cv_done.notify_all(); }
        }
        bool any_busy = false;
        for (Lane& L : S->lanes) any_busy |= L.busy;
        if (S->stop && S->pending.empty() && !any_busy) break;
        if (!progressed) {
            if (any_busy) {
                lk.unlock();                    // poll the device without holding the lock
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            }
        }
    }
}

static void server_destroy(ps_server* S) {
    for (Lane& L : S->lanes) {
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.h_in) (void)hipHostFree(L.h_in);
        if (L.h_out) (void)hipHostFree(L.h_out);
        if (L.h_hdr) (void)hipHostFree(L.h_hdr);
    }
    for (auto& kv : S->all) delete kv.second;
    delete S;
}

extern "C" int ps_server_create(ps_index* ix, const ps_device* pool, const ps_search_params* params,
                                uint64_t run_spectra, uint64_t run_peaks, uint32_t max_runs,
                                uint64_t max_committed_bytes, ps_server** out) {
    if (!out) return fail(PS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ix || !pool || !params) return fail(PS_EINVAL, "NULL argument");
    if (run_spectra == 0 || run_peaks == 0) return fail(PS_EINVAL, "run_spectra and run_peaks must be positive");
    if (max_runs < 1 || max_runs > 64) return fail(PS_EINVAL, "max_runs must be 1..64");
    int rc = require_device();
    if (rc != PS_OK) return rc;
    if (!ix->on_device) return fail(PS_EINVAL, "index is not uploaded");
    if (!pool->base || ((uintptr_t)pool->base & 255u)) return fail(PS_EINVAL, "pool must be a 256-byte aligned block");
    ps_server* S = new (std::nothrow) ps_server();
    if (!S) return fail(PS_ENOMEM, "out of host memory");
    S->ix = ix;
    S->prm = *params;
    S->sc = ix->sched;
    rc = make_kparams(ix, params, &S->kp, &S->sc);
    if (rc != PS_OK) { delete S; return rc; }
    S->pool = (char*)pool->base;
    S->arena = Arena(pool->bytes);
    S->run_n = run_spectra;
    S->run_nnz = run_peaks;
    S->limit = max_committed_bytes ? max_committed_bytes : pool->bytes;
    if (run_bytes(S, 1, PS_MAX_PEAKS_IN) > S->arena.size()) {
        delete S;
        return fail(PS_ENOMEM, "pool of %llu bytes cannot hold a one-spectrum search", (unsigned long long)pool->bytes);
    }
    S->lanes.resize(max_runs);
    hipError_t e = hipSuccess;
    for (Lane& L : S->lanes) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void**)&L.h_hdr, sizeof(BatchHdr), hipHostMallocDefault);
    }
    if (e != hipSuccess) { server_destroy(S); return fail(PS_EDEVICE, "server set-up: %s", hipGetErrorString(e)); }
    S->sched = std::thread(scheduler, S);
    *out = S;
    return PS_OK;
}

extern "C" int ps_server_submit(ps_server* S, const ps_spectra* sp, uint64_t* ticket) {
    if (!S || !sp || !ticket) return fail(PS_EINVAL, "NULL argument");
    int rc = validate_host_spectra(sp, S->kp);
    if (rc != PS_OK) return rc;
    const uint64_t n = sp->n, nnz = n ? sp->peak_off[n] : 0;
    if (n == 0) return fail(PS_EINVAL, "empty request");
    if (n >= (1ull << 31)) return fail(PS_EINVAL, "too many spectra in one request");
    const uint64_t need = run_bytes(S, n, nnz);
    if (need > S->arena.size() || need > S->limit)
        return fail(PS_ENOMEM, "a request of %llu spectra needs %llu device bytes; the server holds %llu",
                    (unsigned long long)n, (unsigned long long)need,
                    (unsigned long long)std::min(S->arena.size(), S->limit));
    {   // refuse early, before copying, when the memory guard is already closed
        std::lock_guard<std::mutex> g(S->mu);
        if (S->committed + need > S->limit) {
            ++S->refused;
            return fail(PS_EAGAIN, "server memory committed (%llu + %llu bytes > %llu); retry later",
                        (unsigned long long)S->committed, (unsigned long long)need, (unsigned long long)S->limit);
        }
    }
    Request* r = new (std::nothrow) Request();
    if (!r) return fail(PS_ENOMEM, "out of host memory");
    try {
        r->off.assign(sp->peak_off, sp->peak_off + n + 1);
        if (nnz) { r->mz.assign(sp->mz, sp->mz + nnz); r->in.assign(sp->intensity, sp->intensity + nnz); }
        r->prec.assign(sp->precursor_mz, sp->precursor_mz + n);
        r->z.assign(sp->charge, sp->charge + n);
    } catch (...) { delete r; return fail(PS_ENOMEM, "out of host memory"); }
    r->need = need;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (S->committed + need > S->limit) {
            ++S->refused;
            delete r;
            return fail(PS_EAGAIN, "server memory committed; retry later");
        }
        S->committed += need;
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
    if (r->claimed) return fail(PS_EINVAL, "ticket %llu is already being waited for", (unsigned long long)ticket);
    r->claimed = true;                 // only this waiter erases and frees the request
    S->cv_done.wait(lk, [&] { return r->done; });
    S->all.erase(ticket);
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
    out->streams = (uint32_t)S->lanes.size();
    out->pool_bytes = S->arena.size();
    out->peak_bytes = S->arena.peak();
    out->committed_bytes = S->committed;
    std::vector<double> v = S->latencies_ms;
    out->samples = v.size();
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
    S->arena.reset_peak();
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
    server_destroy(S);
}

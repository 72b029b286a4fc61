// plan.cpp -- reusable search plans: buffers for a batch capacity and the whole
// kernel sequence of a search captured once as a hipGraph, replayed per batch.
//
// The kernels read the actual batch size from device memory (BatchHdr), so one
// captured graph serves every batch up to the plan's capacity.  Host<->device
// copies stay outside the graph and move exactly the batch's bytes.
#include "batch.h"

#include <cstring>
#include <vector>

using namespace ps;

struct ps_plan {
    ps_index* ix = nullptr;
    KParams kp{};
    Schedule sched{};
    int schedule = PS_SCHED_PERSISTENT;
    bool want_hist = false;
    uint64_t n_cap = 0, nnz_cap = 0, max_items = 0;
    Work w{};
    DevSpectra dsp{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_events = false;          // scan start/end events recorded inside the graph
    hipEvent_t ev_scan0 = nullptr, ev_scan1 = nullptr, ev_start = nullptr, ev_kern = nullptr, ev_done = nullptr;
    BatchHdr* h_hdr = nullptr;
    char* h_stage = nullptr;
    ps_hit* h_hits = nullptr;
    ps_stat* h_stats = nullptr;
    int32_t* h_hist = nullptr;
    unsigned long long* h_counters = nullptr;
    uint64_t n = 0, nnz = 0;
    bool in_flight = false;
};

static void plan_destroy(ps_plan* P) {
    if (!P) return;
    if (P->ev_done && P->in_flight) (void)hipEventSynchronize(P->ev_done);
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    for (hipEvent_t e : {P->ev_scan0, P->ev_scan1, P->ev_start, P->ev_kern, P->ev_done})
        if (e) (void)hipEventDestroy(e);
    for (void* h : {(void*)P->h_hdr, (void*)P->h_stage, (void*)P->h_hits, (void*)P->h_stats, (void*)P->h_hist,
                    (void*)P->h_counters})
        if (h) (void)hipHostFree(h);
    if (P->own_stream && P->stream) (void)hipStreamDestroy(P->stream);
    delete P;
}

static uint64_t stage_bytes(uint64_t n, uint64_t nnz) { return (n + 1) * 8 + nnz * 8 + n * 8 + n; }

extern "C" int ps_plan_bytes(const ps_index* ix, uint64_t n_cap, uint64_t nnz_cap, const ps_search_params* params,
                             uint64_t* bytes) {
    if (!ix || !bytes) return fail(PS_EINVAL, "NULL argument");
    Schedule sc = ix->sched;
    KParams kp;
    int rc = make_kparams(ix, params, &kp, &sc);
    if (rc != PS_OK) return rc;
    *bytes = layout_work(n_cap, nnz_cap, kp, true, max_items_for(ix, n_cap, kp, sc, params->schedule), nullptr,
                         nullptr, nullptr, 0);
    return PS_OK;
}

extern "C" int ps_plan_create(ps_index* ix, const ps_device* work, uint64_t n_cap, uint64_t nnz_cap,
                              const ps_search_params* params, ps_plan** out) {
    if (!out) return fail(PS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ix || !work) return fail(PS_EINVAL, "NULL argument");
    if (n_cap == 0 || n_cap >= (1ull << 31)) return fail(PS_EINVAL, "n_cap must be 1..2^31-1");
    int rc = require_device();
    if (rc != PS_OK) return rc;
    if (!ix->on_device) return fail(PS_EINVAL, "index is not uploaded");
    Schedule sc = ix->sched;
    KParams kp;
    rc = make_kparams(ix, params, &kp, &sc);
    if (rc != PS_OK) return rc;
    const uint64_t max_items = max_items_for(ix, n_cap, kp, sc, params->schedule);
    const uint64_t need = layout_work(n_cap, nnz_cap, kp, true, max_items, nullptr, nullptr, nullptr, 0);
    if (!work->base || work->bytes < need)
        return fail(PS_ENOMEM, "plan needs %llu device bytes, block has %llu", (unsigned long long)need,
                    (unsigned long long)work->bytes);
    if (((uintptr_t)work->base & 255u) != 0) return fail(PS_EINVAL, "device block must be 256-byte aligned");
    ps_plan* P = new (std::nothrow) ps_plan();
    if (!P) return fail(PS_ENOMEM, "out of host memory");
    P->ix = ix; P->kp = kp; P->sched = sc; P->schedule = params->schedule; P->want_hist = params->want_hist != 0;
    P->n_cap = n_cap; P->nnz_cap = nnz_cap; P->max_items = max_items;
    layout_work(n_cap, nnz_cap, kp, true, max_items, (char*)work->base, &P->w, &P->dsp, 0);
    P->dsp.hdr = P->w.hdr;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    if (work->stream) {
        P->stream = (hipStream_t)work->stream;
    } else {
        // a graph cannot be captured on the null stream
        chk(hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking));
        P->own_stream = true;
    }
    for (hipEvent_t* ev : {&P->ev_scan0, &P->ev_scan1, &P->ev_start, &P->ev_kern}) chk(hipEventCreate(ev));
    chk(hipEventCreateWithFlags(&P->ev_done, hipEventBlockingSync));
    chk(hipHostMalloc((void**)&P->h_hdr, sizeof(BatchHdr), hipHostMallocDefault));
    chk(hipHostMalloc((void**)&P->h_stage, stage_bytes(n_cap, nnz_cap), hipHostMallocDefault));
    chk(hipHostMalloc((void**)&P->h_hits, n_cap * kp.top_k * sizeof(ps_hit), hipHostMallocDefault));
    chk(hipHostMalloc((void**)&P->h_stats, n_cap * sizeof(ps_stat), hipHostMallocDefault));
    if (P->want_hist) chk(hipHostMalloc((void**)&P->h_hist, n_cap * (uint64_t)kHistBins * 4, hipHostMallocDefault));
    chk(hipHostMalloc((void**)&P->h_counters, kNumCounters * 8, hipHostMallocDefault));
    if (e != hipSuccess) { plan_destroy(P); return fail(PS_EDEVICE, "plan set-up: %s", hipGetErrorString(e)); }
    // capture the kernel sequence once (with scan events if the runtime records them in graphs)
    for (int attempt = 0; attempt < 2; ++attempt) {
        const bool with_events = attempt == 0;
        e = hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal);
        hipError_t ek = hipSuccess;
        if (e == hipSuccess)
            ek = enqueue_kernels(ix, P->dsp, kp, sc, P->schedule, P->w, false, P->stream,
                                 with_events ? P->ev_scan0 : nullptr, with_events ? P->ev_scan1 : nullptr);
        hipGraph_t g = nullptr;
        hipError_t ee = e == hipSuccess ? hipStreamEndCapture(P->stream, &g) : e;
        if (e == hipSuccess && ek == hipSuccess && ee == hipSuccess && g) {
            e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
            if (e == hipSuccess) { P->graph = g; P->graph_events = with_events; break; }
        }
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        e = ek != hipSuccess ? ek : (ee != hipSuccess ? ee : e);
    }
    if (!P->exec) { plan_destroy(P); return fail(PS_EDEVICE, "graph capture failed: %s", hipGetErrorString(e)); }
    *out = P;
    return PS_OK;
}

static int plan_wait(ps_plan* P) {
    if (!P->in_flight) return PS_OK;
    hipError_t e = hipEventSynchronize(P->ev_done);
    if (e != hipSuccess) return fail(PS_EDEVICE, "plan run failed: %s", hipGetErrorString(e));
    P->in_flight = false;
    return PS_OK;
}

// Replay: header copy, graph, result copies, done event.
static int plan_launch(ps_plan* P) {
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    hipStream_t st = P->stream;
    P->h_hdr->n = P->n;
    P->h_hdr->nnz = P->nnz;
    chk(hipMemcpyAsync(P->w.hdr, P->h_hdr, sizeof(BatchHdr), hipMemcpyHostToDevice, st));
    chk(hipEventRecord(P->ev_start, st));
    chk(hipGraphLaunch(P->exec, st));
    chk(hipEventRecord(P->ev_kern, st));
    if (P->n) {
        chk(hipMemcpyAsync(P->h_hits, P->w.hits, P->n * P->kp.top_k * sizeof(ps_hit), hipMemcpyDeviceToHost, st));
        chk(hipMemcpyAsync(P->h_stats, P->w.stats, P->n * sizeof(ps_stat), hipMemcpyDeviceToHost, st));
        if (P->want_hist)
            chk(hipMemcpyAsync(P->h_hist, P->w.hist, P->n * (uint64_t)kHistBins * 4, hipMemcpyDeviceToHost, st));
    }
    chk(hipMemcpyAsync(P->h_counters, P->w.counters, kNumCounters * 8, hipMemcpyDeviceToHost, st));
    chk(hipEventRecord(P->ev_done, st));
    if (e != hipSuccess) {
        // whatever was enqueued may still use the pinned buffers: let it end
        (void)hipStreamSynchronize(st);
        return fail(PS_EDEVICE, "plan launch: %s", hipGetErrorString(e));
    }
    P->in_flight = true;
    return PS_OK;
}

extern "C" int ps_plan_run(ps_plan* P, const ps_spectra* sp) {
    if (!P || !sp) return fail(PS_EINVAL, "NULL argument");
    int rc = plan_wait(P);
    if (rc != PS_OK) return rc;
    rc = validate_host_spectra(sp, P->kp);
    if (rc != PS_OK) return rc;
    const uint64_t n = sp->n, nnz = n ? sp->peak_off[n] : 0;
    if (n > P->n_cap || nnz > P->nnz_cap)
        return fail(PS_EINVAL, "batch of %llu spectra / %llu peaks exceeds the plan's %llu / %llu",
                    (unsigned long long)n, (unsigned long long)nnz, (unsigned long long)P->n_cap,
                    (unsigned long long)P->nnz_cap);
    P->n = n; P->nnz = nnz;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    if (n) {
        char* h = P->h_stage;
        const uint64_t o_mz = (n + 1) * 8, o_in = o_mz + nnz * 4, o_pr = o_in + nnz * 4, o_z = o_pr + n * 8;
        memcpy(h, sp->peak_off, (n + 1) * 8);
        if (nnz) { memcpy(h + o_mz, sp->mz, nnz * 4); memcpy(h + o_in, sp->intensity, nnz * 4); }
        memcpy(h + o_pr, sp->precursor_mz, n * 8);
        memcpy(h + o_z, sp->charge, n);
        hipStream_t st = P->stream;
        chk(hipMemcpyAsync((void*)P->dsp.peak_off, h, (n + 1) * 8, hipMemcpyHostToDevice, st));
        if (nnz) {
            chk(hipMemcpyAsync((void*)P->dsp.mz, h + o_mz, nnz * 4, hipMemcpyHostToDevice, st));
            chk(hipMemcpyAsync((void*)P->dsp.inten, h + o_in, nnz * 4, hipMemcpyHostToDevice, st));
        }
        chk(hipMemcpyAsync((void*)P->dsp.prec, h + o_pr, n * 8, hipMemcpyHostToDevice, st));
        chk(hipMemcpyAsync((void*)P->dsp.charge, h + o_z, n, hipMemcpyHostToDevice, st));
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(st);              // copies already queued read the staging buffer
            return fail(PS_EDEVICE, "plan input copy: %s", hipGetErrorString(e));
        }
    }
    return plan_launch(P);
}

extern "C" int ps_plan_inputs(ps_plan* P, ps_spectra* dev) {
    if (!P || !dev) return fail(PS_EINVAL, "NULL argument");
    dev->n = P->n_cap;
    dev->peak_off = P->dsp.peak_off; dev->mz = P->dsp.mz; dev->intensity = P->dsp.inten;
    dev->precursor_mz = P->dsp.prec; dev->charge = P->dsp.charge;
    return PS_OK;
}

extern "C" int ps_plan_run_device(ps_plan* P, uint64_t n, uint64_t nnz) {
    if (!P) return fail(PS_EINVAL, "NULL plan");
    int rc = plan_wait(P);
    if (rc != PS_OK) return rc;
    if (n > P->n_cap || nnz > P->nnz_cap) return fail(PS_EINVAL, "batch exceeds the plan's capacity");
    P->n = n; P->nnz = nnz;
    return plan_launch(P);
}

extern "C" int ps_plan_results(ps_plan* P, ps_hit* hits, ps_stat* stats, int32_t* hist) {
    if (!P) return fail(PS_EINVAL, "NULL plan");
    int rc = plan_wait(P);
    if (rc != PS_OK) return rc;
    const uint64_t n = P->n;
    if (hits) memcpy(hits, P->h_hits, n * P->kp.top_k * sizeof(ps_hit));
    if (stats) memcpy(stats, P->h_stats, n * sizeof(ps_stat));
    if (hist) {
        if (!P->want_hist) return fail(PS_EINVAL, "plan was made without want_hist");
        memcpy(hist, P->h_hist, n * (uint64_t)kHistBins * 4);
    }
    for (uint64_t i = 0; i < n; ++i)
        if (P->h_stats[i].status == PS_STATUS_OVERFLOW)
            return fail(PS_EOVERFLOW, "spectrum %llu exceeded the shared-peak counter bounds", (unsigned long long)i);
    return PS_OK;
}

extern "C" int ps_plan_timing(ps_plan* P, double* graph_ms, double* scan_ms, uint64_t* postings, uint64_t* lookups,
                              uint64_t* items) {
    if (!P) return fail(PS_EINVAL, "NULL plan");
    int rc = plan_wait(P);
    if (rc != PS_OK) return rc;
    float g = 0.0f, s = -1.0f;
    hipError_t e = hipEventElapsedTime(&g, P->ev_start, P->ev_kern);
    if (e != hipSuccess) return fail(PS_EDEVICE, "event timing: %s", hipGetErrorString(e));
    if (P->graph_events && hipEventElapsedTime(&s, P->ev_scan0, P->ev_scan1) != hipSuccess) {
        (void)hipGetLastError();
        s = -1.0f;
    }
    if (graph_ms) *graph_ms = g;
    if (scan_ms) *scan_ms = s;
    if (postings) *postings = P->h_counters[kCtrPostings];
    if (lookups) *lookups = P->h_counters[kCtrLookups];
    if (items) *items = P->h_counters[kCtrItems];
    return PS_OK;
}

extern "C" int ps_plan_counters(ps_plan* P, ps_counters* out) {
    if (!P || !out) return fail(PS_EINVAL, "NULL argument");
    int rc = plan_wait(P);
    if (rc != PS_OK) return rc;
    memset(out, 0, sizeof *out);
    const unsigned long long* c = P->h_counters;
    out->postings = c[kCtrPostings];
    out->bin_lookups = c[kCtrLookups];
    out->work_items = P->schedule == PS_SCHED_PERSISTENT ? c[kCtrItems] : 0;
    out->wide_spectra = c[kCtrWide];
    out->overflow_spectra = c[kCtrOverflow];
    out->dense_postings = c[kCtrDensePost];
    out->dense_reads = c[kCtrDenseIds];
    return PS_OK;
}

extern "C" int ps_plan_device_results(ps_plan* P, ps_hit** hits, ps_stat** stats, int32_t** hist) {
    if (!P) return fail(PS_EINVAL, "NULL plan");
    if (hits) *hits = P->w.hits;
    if (stats) *stats = P->w.stats;
    if (hist) *hist = P->w.hist;
    return PS_OK;
}

extern "C" int ps_plan_stream(ps_plan* P, void** stream) {
    if (!P || !stream) return fail(PS_EINVAL, "NULL argument");
    *stream = P->stream;
    return PS_OK;
}

// 1 when the plan is idle or its run has finished, 0 while it runs, -1 on error.
extern "C" int ps_plan_event_query(ps_plan* P) {
    if (!P || !P->in_flight) return 1;
    hipError_t e = hipEventQuery(P->ev_done);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return -1;
}

extern "C" void ps_plan_free(ps_plan* P) { plan_destroy(P); }

// capi.cpp -- the C ABI: errors, batches, launches and results.
#include "state.h"
#include "batch.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

namespace ps {

static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

static int g_cu_count = 0;

int device_cu_count() { return g_cu_count > 0 ? g_cu_count : 256; }

int require_device() {
    static std::once_flag once;
    static int state = PS_EDEVICE;
    static std::string msg;
    std::call_once(once, [] {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || n == 0) { msg = "no HIP device available"; return; }
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            msg = "cannot query the HIP device";
            return;
        }
        if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            msg = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950 only";
            return;
        }
        g_cu_count = prop.multiProcessorCount;
        hipError_t ea = init_kernel_attributes();
        if (ea != hipSuccess) { msg = std::string("kernel set-up: ") + hipGetErrorString(ea); return; }
        state = PS_OK;
    });
    if (state != PS_OK) return fail(state, "%s", msg.c_str());
    return PS_OK;
}

static uint64_t a256(uint64_t x) { return (x + 255) & ~255ull; }

// Validate search parameters and derive the kernel view.
int make_kparams(const ps_index* ix, const ps_search_params* p, KParams* kp, const Schedule* sched) {
    if (!p) return fail(PS_EINVAL, "params is NULL");
    if (p->top_k < 1 || p->top_k > PS_MAX_TOP_K) return fail(PS_EINVAL, "top_k must be 1..%d", PS_MAX_TOP_K);
    if (p->top_peaks < 1 || p->top_peaks > PS_MAX_TOP_PEAKS)
        return fail(PS_EINVAL, "top_peaks must be 1..%d", PS_MAX_TOP_PEAKS);
    if (p->min_shared < 1) return fail(PS_EINVAL, "min_shared must be >= 1");
    if (p->frag_tol_bins < 0 || p->frag_tol_bins > PS_MAX_FRAG_TOL_BINS)
        return fail(PS_EINVAL, "frag_tol_bins must be 0..%d", PS_MAX_FRAG_TOL_BINS);
    if (p->window < 0) return fail(PS_EINVAL, "window must be >= 0");
    if (p->window_is_ppm && p->window > 1000000) return fail(PS_EINVAL, "ppm window must be <= 1e6");
    if (!p->window_is_ppm && p->window > (1ll << 60)) return fail(PS_EINVAL, "window too large");
    if (p->max_charge < 1 || p->max_charge > PS_MAX_CHARGE)
        return fail(PS_EINVAL, "max_charge must be 1..%d", PS_MAX_CHARGE);
    if (p->schedule != PS_SCHED_PLAIN && p->schedule != PS_SCHED_PERSISTENT)
        return fail(PS_EINVAL, "unknown schedule %d", p->schedule);
    if (p->fit != PS_FIT_TAIL && p->fit != PS_FIT_GUMBEL) return fail(PS_EINVAL, "unknown fit %d", p->fit);
    if (p->noise_permille > 1000) return fail(PS_EINVAL, "noise_permille must be 0..1000");
    if (p->intensity != PS_INTENSITY_LINEAR && p->intensity != PS_INTENSITY_SQRT)
        return fail(PS_EINVAL, "unknown intensity normalisation %d", p->intensity);
    if (p->reserved != 0) return fail(PS_EINVAL, "reserved must be 0");
    const uint32_t cmax = p->max_charge > 2 ? p->max_charge - 1 : 1;
    const uint64_t stride = (uint64_t)p->top_peaks * cmax;
    if (ix && ix->merge_tol && (uint32_t)p->frag_tol_bins != ix->merge_tol)
        return fail(PS_EINVAL, "this index merges the lists of %u neighbouring bins; search with frag_tol_bins = %u",
                    ix->merge_tol, ix->merge_tol);
    // probes per entry: 2T+1 bins, or the one merged list
    const uint64_t width = (ix && ix->merge_tol) ? 1 : (uint64_t)(2 * p->frag_tol_bins + 1);
    const uint64_t segs = stride * width;
    if (segs > PS_MAX_SEGMENTS)
        return fail(PS_EINVAL, "top_peaks * max(1, max_charge-1) * probes per peak = %llu exceeds %d",
                    (unsigned long long)segs, PS_MAX_SEGMENTS);
    kp->window = p->window;
    kp->window_is_ppm = p->window_is_ppm ? 1 : 0;
    kp->tol = p->frag_tol_bins;
    kp->top_peaks = p->top_peaks;
    kp->top_k = p->top_k;
    kp->min_shared = p->min_shared;
    kp->max_charge = p->max_charge;
    kp->ent_stride = (uint32_t)stride;
    kp->seg_cap = (uint32_t)segs;
    kp->fit = p->fit;
    kp->noise_permille = p->noise_permille;
    kp->intensity = p->intensity;
    int rc = check_schedule(*sched);
    if (rc != PS_OK) return rc;
    if (ix && sched->tile < (1u << ix->dir_shift))
        return fail(PS_EINVAL, "tile %u is smaller than this index's tile grain %u", sched->tile,
                    1u << ix->dir_shift);
    kp->tile = sched->tile;
    kp->tile_shift = (uint32_t)__builtin_ctz(sched->tile);
    kp->nt = sched->group_threads ? sched->group_threads : 256;
    if (scan_lds_bytes(*kp, false) > kMaxLds)
        return fail(PS_EINVAL, "tile %u needs %zu bytes of LDS with these parameters (max %zu)", kp->tile,
                    scan_lds_bytes(*kp, false), kMaxLds);
    return PS_OK;
}

Schedule default_schedule() {
    Schedule s{};
    s.tile = 4096;
    s.tiles_per_item = 64;
    s.groups_per_cu = 6;
    return s;
}

int check_schedule(const Schedule& s) {
    if (s.tile < 1024 || s.tile > 32768 || (s.tile & (s.tile - 1)))
        return fail(PS_EINVAL, "tile must be a power of two in 1024..32768");
    if (s.group_threads != 0 && s.group_threads != 256 && s.group_threads != 512)
        return fail(PS_EINVAL, "group_threads must be 256 or 512 (0 means 256)");
    if (s.group_threads == 512 && s.tile < 8192)
        return fail(PS_EINVAL, "512-thread workgroups need tiles of at least 8192 candidates");
    if (s.tiles_per_item < 1 || s.tiles_per_item > 4096) return fail(PS_EINVAL, "tiles_per_item must be 1..4096");
    if (s.groups_per_cu < 1 || s.groups_per_cu > 8) return fail(PS_EINVAL, "groups_per_cu must be 1..8");
    for (uint32_t r : s.reserved)
        if (r) return fail(PS_EINVAL, "reserved schedule fields must be 0");
    return PS_OK;
}

// Carve the batch workspace out of the caller's block.  Returns bytes needed.
uint64_t layout_work(uint64_t n, uint64_t nnz, const KParams& kp, bool copy_inputs, uint64_t max_items,
                     char* base, Work* w, DevSpectra* dsp, uint64_t dump_cap) {
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) { uint64_t at = o; o = a256(o + bytes); return base ? base + at : nullptr; };
    if (copy_inputs) {
        char* p_off = take((n + 1) * 8);
        char* p_mz = take(nnz * 4);
        char* p_in = take(nnz * 4);
        char* p_pr = take(n * 8);
        char* p_z = take(n);
        if (dsp) {
            dsp->peak_off = (const uint64_t*)p_off; dsp->mz = (const float*)p_mz; dsp->inten = (const float*)p_in;
            dsp->prec = (const double*)p_pr; dsp->charge = (const int8_t*)p_z; dsp->n = n; dsp->nnz = nnz;
        }
    }
    Work t;
    memset(&t, 0, sizeof t);
    t.hdr = (BatchHdr*)take(sizeof(BatchHdr));
    t.entries = (uint32_t*)take(n * (uint64_t)kp.ent_stride * 4);
    t.info = (SpecInfo*)take(n * sizeof(SpecInfo));
    t.hist = (int32_t*)take(n * (uint64_t)kHistBins * 4);
    t.n_scored = (unsigned long long*)take(n * 8);
    t.partial = (ps_hit*)take(max_items * (uint64_t)kp.top_k * sizeof(ps_hit));
    t.spec_item0 = (uint32_t*)take((n + 1) * 4);
    t.hits = (ps_hit*)take(n * (uint64_t)kp.top_k * sizeof(ps_hit));
    t.stats = (ps_stat*)take(n * sizeof(ps_stat));
    t.counters = (unsigned long long*)take(kNumCounters * 8);
    if (dump_cap) {
        t.dump_spec = (uint32_t*)take(dump_cap * 4);
        t.dump_id = (uint32_t*)take(dump_cap * 4);
        t.dump_cnt_lo = (uint32_t*)take(dump_cap * 4);
        t.dump_cnt_hi = (uint32_t*)take(dump_cap * 4);
        t.dump_cap = dump_cap;
    }
    if (w) *w = t;
    return o;
}

// Upper bound on persistent work items: every spectrum's window split into
// items of tiles_per_item tiles.
uint64_t max_items_for(const ps_index* ix, uint64_t n, const KParams& kp, const Schedule& sc, int schedule) {
    if (schedule == PS_SCHED_PLAIN) return n;
    uint64_t span = (uint64_t)kp.tile * sc.tiles_per_item;
    uint64_t per = ix->n_entries / span + 2;    // grid-aligned items touching one window
    return n * per;
}

int validate_host_spectra(const ps_spectra* sp, const KParams& kp) {
    if (!sp) return fail(PS_EINVAL, "spectra is NULL");
    if (sp->n && (!sp->peak_off || !sp->precursor_mz || !sp->charge)) return fail(PS_EINVAL, "NULL spectra array");
    if (sp->n == 0) return PS_OK;
    if (sp->peak_off[0] != 0) return fail(PS_EINVAL, "peak_off[0] must be 0");
    const uint64_t nnz = sp->peak_off[sp->n];
    if (nnz && (!sp->mz || !sp->intensity)) return fail(PS_EINVAL, "NULL peak arrays");
    for (uint64_t i = 0; i < sp->n; ++i) {
        uint64_t a = sp->peak_off[i], b = sp->peak_off[i + 1];
        if (b < a) return fail(PS_EINVAL, "spectrum %llu: peak_off decreases", (unsigned long long)i);
        if (b - a > PS_MAX_PEAKS_IN)
            return fail(PS_EINVAL, "spectrum %llu has %llu peaks (max %d)", (unsigned long long)i,
                        (unsigned long long)(b - a), PS_MAX_PEAKS_IN);
        int z = sp->charge[i];
        if (z < 1 || z > (int)kp.max_charge)
            return fail(PS_EINVAL, "spectrum %llu: charge %d outside 1..%u", (unsigned long long)i, z, kp.max_charge);
        double pm = sp->precursor_mz[i];
        if (!(pm > 0.0) || !(pm <= 1e6)) return fail(PS_EINVAL, "spectrum %llu: bad precursor m/z", (unsigned long long)i);
        if ((double)z * (pm * 1e6) < (double)z * (double)kProtonUda)
            return fail(PS_EINVAL, "spectrum %llu: precursor below one proton", (unsigned long long)i);
    }
    for (uint64_t j = 0; j < nnz; ++j) {
        float m = sp->mz[j], v = sp->intensity[j];
        if (!(m > 0.0f) || !std::isfinite(m) || !(v >= 0.0f) || !std::isfinite(v))
            return fail(PS_EINVAL, "peak %llu: m/z must be finite > 0 and intensity finite >= 0",
                        (unsigned long long)j);
    }
    return PS_OK;
}

// Kernel sequence of one search (no host copies): zero the accumulators,
// prep + window, scan (plain or persistent), merge + expect values.  Reads the
// batch size from w.hdr, so it can be captured once and replayed.
hipError_t enqueue_kernels(const ps_index* ix, const DevSpectra& dsp, const KParams& kp, const Schedule& sc,
                           int schedule, const Work& w, bool dump, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(launch_fill_per_spectrum(w.hist, 0, (uint64_t)kHistBins, dsp.n * (uint64_t)kHistBins, w.hdr, st));
    chk(launch_fill_per_spectrum(w.n_scored, 0, 2, dsp.n * 2, w.hdr, st));
    chk(launch_fill_u32(w.counters, 0, 2 * kNumCounters, st));
    chk(launch_prep(ix->dev, dsp, kp, w, st));
    if (ev0) chk(hipEventRecord(ev0, st));
    const bool per_item = schedule == PS_SCHED_PERSISTENT;
    if (per_item) {
        chk(launch_worklist(dsp, kp, w, sc.tiles_per_item, st));
        const uint32_t grid = (uint32_t)device_cu_count() * sc.groups_per_cu;
        chk(launch_scan_persistent(ix->dev, dsp, kp, w, grid, sc.tiles_per_item, st));
    } else {
        chk(launch_scan_plain(ix->dev, dsp, kp, w, dump, false, false, st));
    }
    if (ev1) chk(hipEventRecord(ev1, st));
    chk(launch_merge(ix->dev, dsp, kp, w, per_item, st));
    return e;
}

// Enqueue the whole search for a batch whose inputs are in device memory.
int enqueue_search(ps_batch* B) {
    hipStream_t st = B->stream;
    const Work& w = B->w;
    const uint64_t n = B->n;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(hipMemcpyAsync(w.hdr, B->h_hdr, sizeof(BatchHdr), hipMemcpyHostToDevice, st));
    chk(enqueue_kernels(B->ix, B->dsp, B->kp, B->sched, B->schedule, w, B->dump, st, B->ev_scan0, B->ev_scan1));
    // results to pinned host memory
    chk(hipMemcpyAsync(B->h_hits, w.hits, n * (uint64_t)B->kp.top_k * sizeof(ps_hit), hipMemcpyDeviceToHost, st));
    chk(hipMemcpyAsync(B->h_stats, w.stats, n * sizeof(ps_stat), hipMemcpyDeviceToHost, st));
    if (B->want_hist) chk(hipMemcpyAsync(B->h_hist, w.hist, n * (uint64_t)kHistBins * 4, hipMemcpyDeviceToHost, st));
    chk(hipMemcpyAsync(B->h_counters, w.counters, kNumCounters * 8, hipMemcpyDeviceToHost, st));
    chk(hipEventRecord(B->ev_done, st));
    if (e != hipSuccess) return fail(PS_EDEVICE, "enqueue: %s", hipGetErrorString(e));
    B->scan_launches = 2;
    return PS_OK;
}

static void batch_destroy(ps_batch* B) {
    if (!B) return;
    if (B->ev_done) { (void)hipEventSynchronize(B->ev_done); (void)hipEventDestroy(B->ev_done); }
    if (B->ev_scan0) (void)hipEventDestroy(B->ev_scan0);
    if (B->ev_scan1) (void)hipEventDestroy(B->ev_scan1);
    if (B->h_hits) (void)hipHostFree(B->h_hits);
    if (B->h_stats) (void)hipHostFree(B->h_stats);
    if (B->h_hist) (void)hipHostFree(B->h_hist);
    if (B->h_counters) (void)hipHostFree(B->h_counters);
    if (B->h_stage) (void)hipHostFree(B->h_stage);
    if (B->h_hdr) (void)hipHostFree(B->h_hdr);
    delete B;
}

// A batch that failed after work was enqueued: that work may still read the
// pinned buffers, so its stream is drained before they are freed.
static void batch_abort(ps_batch* B) {
    (void)hipStreamSynchronize(B->stream);
    batch_destroy(B);
}

// Common batch set-up; inputs either copied from host (host_sp) or device-resident (dev_sp).
int batch_begin(ps_index* ix, const ps_device* work, const ps_spectra* host_sp, const ps_spectra* dev_sp,
                uint64_t dev_nnz, const ps_search_params* params, uint64_t dump_cap, ps_batch** out) {
    if (!out) return fail(PS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ix || !work) return fail(PS_EINVAL, "NULL argument");
    int rc = require_device();
    if (rc != PS_OK) return rc;
    if (!ix->on_device) return fail(PS_EINVAL, "index is not uploaded");
    Schedule sc = ix->sched;
    KParams kp;
    rc = make_kparams(ix, params, &kp, &sc);
    if (rc != PS_OK) return rc;
    const ps_spectra* sp = host_sp ? host_sp : dev_sp;
    if (host_sp) { rc = validate_host_spectra(host_sp, kp); if (rc != PS_OK) return rc; }
    else if (!dev_sp) return fail(PS_EINVAL, "spectra is NULL");
    const uint64_t n = sp->n;
    const uint64_t nnz = host_sp ? (n ? host_sp->peak_off[n] : 0) : dev_nnz;
    if (n >= (1ull << 31)) return fail(PS_EINVAL, "too many spectra in one batch");
    const uint64_t max_items = max_items_for(ix, n, kp, sc, params->schedule);
    uint64_t need = layout_work(n, nnz, kp, host_sp != nullptr, max_items, nullptr, nullptr, nullptr, dump_cap);
    if (!work->base || work->bytes < need)
        return fail(PS_ENOMEM, "batch needs %llu device bytes, block has %llu", (unsigned long long)need,
                    (unsigned long long)work->bytes);
    if (((uintptr_t)work->base & 255u) != 0) return fail(PS_EINVAL, "device block must be 256-byte aligned");
    ps_batch* B = new (std::nothrow) ps_batch();
    if (!B) return fail(PS_ENOMEM, "out of host memory");
    B->ix = ix; B->n = n; B->kp = kp; B->sched = sc; B->schedule = params->schedule;
    B->want_hist = params->want_hist != 0; B->stream = (hipStream_t)work->stream; B->max_items = max_items;
    B->dump = dump_cap != 0;
    DevSpectra dsp;
    layout_work(n, nnz, kp, host_sp != nullptr, max_items, (char*)work->base, &B->w, &dsp, dump_cap);
    if (!host_sp) {
        dsp.peak_off = dev_sp->peak_off; dsp.mz = dev_sp->mz; dsp.inten = dev_sp->intensity;
        dsp.prec = dev_sp->precursor_mz; dsp.charge = dev_sp->charge; dsp.n = n; dsp.nnz = nnz;
    }
    dsp.hdr = B->w.hdr;
    B->dsp = dsp;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(hipEventCreate(&B->ev_scan0));
    chk(hipEventCreate(&B->ev_scan1));
    chk(hipEventCreateWithFlags(&B->ev_done, hipEventBlockingSync));
    const uint64_t nh = std::max<uint64_t>(n, 1);
    chk(hipHostMalloc((void**)&B->h_hits, nh * kp.top_k * sizeof(ps_hit), hipHostMallocDefault));
    chk(hipHostMalloc((void**)&B->h_stats, nh * sizeof(ps_stat), hipHostMallocDefault));
    if (B->want_hist) chk(hipHostMalloc((void**)&B->h_hist, nh * (uint64_t)kHistBins * 4, hipHostMallocDefault));
    chk(hipHostMalloc((void**)&B->h_counters, kNumCounters * 8, hipHostMallocDefault));
    chk(hipHostMalloc((void**)&B->h_hdr, sizeof(BatchHdr), hipHostMallocDefault));
    if (e == hipSuccess) { B->h_hdr->n = n; B->h_hdr->nnz = nnz; }
    if (e != hipSuccess) { batch_destroy(B); return fail(PS_EDEVICE, "batch set-up: %s", hipGetErrorString(e)); }
    if (host_sp && n) {
        // stage inputs in pinned memory, then copy on the batch's stream
        const uint64_t bytes = (n + 1) * 8 + nnz * 8 + n * 8 + n;
        chk(hipHostMalloc((void**)&B->h_stage, bytes, hipHostMallocDefault));
        if (e == hipSuccess) {
            char* h = B->h_stage;
            memcpy(h, host_sp->peak_off, (n + 1) * 8);
            memcpy(h + (n + 1) * 8, host_sp->mz, nnz * 4);
            memcpy(h + (n + 1) * 8 + nnz * 4, host_sp->intensity, nnz * 4);
            memcpy(h + (n + 1) * 8 + nnz * 8, host_sp->precursor_mz, n * 8);
            memcpy(h + (n + 1) * 8 + nnz * 8 + n * 8, host_sp->charge, n);
            chk(hipMemcpyAsync((void*)dsp.peak_off, h, (n + 1) * 8, hipMemcpyHostToDevice, B->stream));
            if (nnz) {
                chk(hipMemcpyAsync((void*)dsp.mz, h + (n + 1) * 8, nnz * 4, hipMemcpyHostToDevice, B->stream));
                chk(hipMemcpyAsync((void*)dsp.inten, h + (n + 1) * 8 + nnz * 4, nnz * 4, hipMemcpyHostToDevice, B->stream));
            }
            chk(hipMemcpyAsync((void*)dsp.prec, h + (n + 1) * 8 + nnz * 8, n * 8, hipMemcpyHostToDevice, B->stream));
            chk(hipMemcpyAsync((void*)dsp.charge, h + (n + 1) * 8 + nnz * 8 + n * 8, n, hipMemcpyHostToDevice, B->stream));
        }
        if (e != hipSuccess) { batch_abort(B); return fail(PS_EDEVICE, "input copy: %s", hipGetErrorString(e)); }
    }
    if (n) {
        rc = enqueue_search(B);
        if (rc != PS_OK) { batch_abort(B); return rc; }
    } else {
        (void)hipEventRecord(B->ev_scan0, B->stream);
        (void)hipEventRecord(B->ev_scan1, B->stream);
        (void)hipEventRecord(B->ev_done, B->stream);
    }
    *out = B;
    return PS_OK;
}

}  // namespace ps

using namespace ps;

extern "C" const char* ps_last_error(void) { return g_err.c_str(); }

extern "C" int ps_workspace_bytes(const ps_index* ix, uint64_t n, uint64_t nnz, const ps_search_params* params,
                                  uint64_t* bytes) {
    if (!ix || !bytes) return fail(PS_EINVAL, "NULL argument");
    Schedule sc = ix->sched;
    KParams kp;
    int rc = make_kparams(ix, params, &kp, &sc);
    if (rc != PS_OK) return rc;
    *bytes = layout_work(n, nnz, kp, true, max_items_for(ix, n, kp, sc, params->schedule), nullptr, nullptr,
                         nullptr, 0);
    return PS_OK;
}

extern "C" int ps_search_batch(ps_index* ix, const ps_device* work, const ps_spectra* spectra,
                               const ps_search_params* params, ps_batch** out) {
    return batch_begin(ix, work, spectra, nullptr, 0, params, 0, out);
}

extern "C" int ps_search_device(ps_index* ix, const ps_device* work, const ps_spectra* spectra, uint64_t nnz,
                                const ps_search_params* params, ps_batch** out) {
    return batch_begin(ix, work, nullptr, spectra, nnz, params, 0, out);
}

extern "C" int ps_results(ps_batch* B, ps_hit* hits, ps_stat* stats, int32_t* hist) {
    if (!B) return fail(PS_EINVAL, "NULL batch");
    hipError_t e = hipEventSynchronize(B->ev_done);
    if (e != hipSuccess) return fail(PS_EDEVICE, "batch failed: %s", hipGetErrorString(e));
    const uint64_t n = B->n;
    if (hits) memcpy(hits, B->h_hits, n * (uint64_t)B->kp.top_k * sizeof(ps_hit));
    if (stats) memcpy(stats, B->h_stats, n * sizeof(ps_stat));
    if (hist) {
        if (!B->want_hist) return fail(PS_EINVAL, "batch was searched without want_hist");
        memcpy(hist, B->h_hist, n * (uint64_t)kHistBins * 4);
    }
    for (uint64_t i = 0; i < n; ++i)
        if (B->h_stats[i].status == PS_STATUS_OVERFLOW)
            return fail(PS_EOVERFLOW, "spectrum %llu exceeded the shared-peak counter bounds", (unsigned long long)i);
    return PS_OK;
}

extern "C" int ps_batch_device_results(ps_batch* B, ps_hit** hits, ps_stat** stats, int32_t** hist) {
    if (!B) return fail(PS_EINVAL, "NULL batch");
    if (hits) *hits = B->w.hits;
    if (stats) *stats = B->w.stats;
    if (hist) *hist = B->w.hist;
    return PS_OK;
}

extern "C" int ps_assemble(void* stream, uint32_t n_shards, const ps_part* parts, uint64_t n, uint32_t top_k,
                           int32_t fit, ps_hit* hits, ps_stat* stats, int32_t* hist) {
    if (n_shards < 1 || n_shards > PS_MAX_SHARDS)
        return fail(PS_EINVAL, "n_shards must be 1..%d", PS_MAX_SHARDS);
    if (top_k < 1 || top_k > PS_MAX_TOP_K) return fail(PS_EINVAL, "top_k must be 1..%d", PS_MAX_TOP_K);
    if (fit != PS_FIT_TAIL && fit != PS_FIT_GUMBEL) return fail(PS_EINVAL, "unknown fit %d", fit);
    if (n == 0) return PS_OK;
    if (!parts || !hits || !stats) return fail(PS_EINVAL, "NULL argument");
    for (uint32_t g = 0; g < n_shards; ++g) {
        if (!parts[g].hits || !parts[g].stats)
            return fail(PS_EINVAL, "partition %u has a NULL result pointer", g);
        if ((parts[g].hist == nullptr) == (parts[g].sampled == nullptr))
            return fail(PS_EINVAL, "partition %u must give exactly one of hist and sampled", g);
    }
    int rc = require_device();
    if (rc != PS_OK) return rc;
    hipError_t e = launch_assemble(parts, n_shards, n, top_k, fit, hits, stats, hist, (hipStream_t)stream);
    if (e != hipSuccess) return fail(PS_EDEVICE, "assemble: %s", hipGetErrorString(e));
    return PS_OK;
}

static_assert(sizeof(ps_sampled) == 256, "a sampled partial result is 256 bytes");

extern "C" int ps_sample(void* stream, uint64_t n, const int32_t* hist, const ps_stat* stats, ps_sampled* out) {
    if (n == 0) return PS_OK;
    if (!hist || !stats || !out) return fail(PS_EINVAL, "NULL argument");
    int rc = require_device();
    if (rc != PS_OK) return rc;
    hipError_t e = launch_sample(hist, stats, out, n, (hipStream_t)stream);
    if (e != hipSuccess) return fail(PS_EDEVICE, "sample: %s", hipGetErrorString(e));
    return PS_OK;
}

extern "C" int ps_batch_timing(ps_batch* B, double* scan_ms, uint32_t* launches, uint64_t* postings,
                               uint64_t* lookups) {
    if (!B) return fail(PS_EINVAL, "NULL batch");
    hipError_t e = hipEventSynchronize(B->ev_done);
    if (e != hipSuccess) return fail(PS_EDEVICE, "batch failed: %s", hipGetErrorString(e));
    float ms = 0.0f;
    if (B->n) {
        e = hipEventElapsedTime(&ms, B->ev_scan0, B->ev_scan1);
        if (e != hipSuccess) return fail(PS_EDEVICE, "event timing: %s", hipGetErrorString(e));
    }
    if (scan_ms) *scan_ms = ms;
    if (launches) *launches = B->scan_launches;
    if (postings) *postings = B->n ? B->h_counters[kCtrPostings] : 0;
    if (lookups) *lookups = B->n ? B->h_counters[kCtrLookups] : 0;
    return PS_OK;
}

extern "C" int ps_batch_counters(ps_batch* B, ps_counters* out) {
    if (!B || !out) return fail(PS_EINVAL, "NULL argument");
    hipError_t e = hipEventSynchronize(B->ev_done);
    if (e != hipSuccess) return fail(PS_EDEVICE, "batch failed: %s", hipGetErrorString(e));
    memset(out, 0, sizeof *out);
    if (B->n) {
        const unsigned long long* c = B->h_counters;
        out->postings = c[kCtrPostings];
        out->bin_lookups = c[kCtrLookups];
        out->work_items = B->schedule == PS_SCHED_PERSISTENT ? c[kCtrItems] : 0;
        out->wide_spectra = c[kCtrWide];
        out->overflow_spectra = c[kCtrOverflow];
        out->dense_postings = c[kCtrDensePost];
        out->dense_reads = c[kCtrDenseIds];
    }
    return PS_OK;
}

extern "C" int ps_search_dump(ps_index* ix, const ps_device* work, const ps_spectra* spectra,
                              const ps_search_params* params, uint64_t cap, uint32_t* spectrum, uint32_t* id,
                              uint16_t* n_b, uint16_t* n_y, uint32_t* sum_q, uint64_t* count) {
    if (!count || cap == 0) return fail(PS_EINVAL, "count is NULL or cap is 0");
    if (params && params->schedule != PS_SCHED_PLAIN) return fail(PS_EINVAL, "dump needs the plain schedule");
    ps_batch* B = nullptr;
    int rc = batch_begin(ix, work, spectra, nullptr, 0, params, cap, &B);
    if (rc != PS_OK) return rc;
    hipError_t e = hipEventSynchronize(B->ev_done);
    if (e != hipSuccess) { batch_destroy(B); return fail(PS_EDEVICE, "dump: %s", hipGetErrorString(e)); }
    uint64_t total = B->n ? B->h_counters[kCtrDump] : 0;
    *count = total;
    uint64_t m = std::min(total, cap);
    std::vector<uint32_t> a(m), b(m), c(m), d(m);
    if (m) {
        e = hipMemcpy(a.data(), B->w.dump_spec, m * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(b.data(), B->w.dump_id, m * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(c.data(), B->w.dump_cnt_lo, m * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(d.data(), B->w.dump_cnt_hi, m * 4, hipMemcpyDeviceToHost);
    }
    batch_destroy(B);
    if (e != hipSuccess) return fail(PS_EDEVICE, "dump copy: %s", hipGetErrorString(e));
    for (uint64_t i = 0; i < m; ++i) {
        if (spectrum) spectrum[i] = a[i];
        if (id) id[i] = b[i];
        if (n_b) n_b[i] = (uint16_t)(c[i] & 0xFFFFu);
        if (n_y) n_y[i] = (uint16_t)(c[i] >> 16);
        if (sum_q) sum_q[i] = d[i];
    }
    return total > cap ? fail(PS_ENOMEM, "dump holds %llu candidates, cap %llu", (unsigned long long)total,
                              (unsigned long long)cap)
                       : PS_OK;
}

extern "C" void ps_batch_free(ps_batch* B) { batch_destroy(B); }

extern "C" int ps_index_set_schedule(ps_index* ix, const ps_schedule* s) {
    if (!ix || !s) return fail(PS_EINVAL, "NULL argument");
    int rc = check_schedule(*s);
    if (rc != PS_OK) return rc;
    if (s->tile < (1u << ix->dir_shift))
        return fail(PS_EINVAL, "tile %u is smaller than this index's tile grain %u", s->tile, 1u << ix->dir_shift);
    ix->sched = *s;
    return PS_OK;
}

extern "C" int ps_index_get_schedule(const ps_index* ix, ps_schedule* s) {
    if (!ix || !s) return fail(PS_EINVAL, "NULL argument");
    *s = ix->sched;
    return PS_OK;
}

// noalloc.cpp -- a search entry point that allocates nothing.
//
// ps_search_static runs the same kernels as ps_search_device, but every
// buffer beyond the caller's inputs and outputs (the batch header, bin
// entries, window summaries, histograms when the caller wants none back,
// scored counts, partial top-k lists, work list and counters) lives in one
// file-scope device array of fixed size.  Each GPU the library runs on holds
// its own copy of the array until the process ends; its device address is
// looked up once per device and kept.  The entry point makes no device or
// pinned host allocation, creates no event and copies nothing from the host:
// the batch size reaches the device through a kernel argument, so the call can
// also be recorded into a graph.
#include "batch.h"

#include <mutex>

namespace {

constexpr uint64_t kStaticScratchBytes = PS_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

// The shared work area of ps_search_static (one per device).
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up on first use.
int scratch_for_current_device(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return ps::fail(PS_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return ps::fail(PS_EDEVICE, "device %d is beyond the %d supported", dev,
                                                       kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return ps::fail(PS_EDEVICE, "static scratch address: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (char*)p;
    }
    *out = g_scratch_ptr[dev];
    return PS_OK;
}

}  // namespace

using namespace ps;

extern "C" int ps_search_static(ps_index* ix, void* stream, const ps_spectra* spectra, uint64_t nnz,
                                const ps_search_params* params, ps_hit* hits, ps_stat* stats, int32_t* hist) {
    if (!ix || !spectra || !params) return fail(PS_EINVAL, "NULL argument");
    const uint64_t n = spectra->n;
    if (n && (!spectra->peak_off || !spectra->precursor_mz || !spectra->charge || !hits || !stats))
        return fail(PS_EINVAL, "NULL spectra or result pointer");
    if (nnz && (!spectra->mz || !spectra->intensity)) return fail(PS_EINVAL, "NULL peak arrays");
    if (n >= (1ull << 31)) return fail(PS_EINVAL, "too many spectra in one batch");
    int rc = require_device();
    if (rc != PS_OK) return rc;
    if (!ix->on_device) return fail(PS_EINVAL, "index is not uploaded");
    Schedule sc = ix->sched;
    KParams kp;
    rc = make_kparams(ix, params, &kp, &sc);
    if (rc != PS_OK) return rc;
    const uint64_t items = max_items_for(ix, n, kp, sc, params->schedule);
    const uint64_t need = layout_work(n, nnz, kp, false, items, nullptr, nullptr, nullptr, 0);
    if (need > kStaticScratchBytes)
        return fail(PS_ENOMEM, "a batch of %llu spectra needs %llu bytes of work area; the static area holds %llu "
                    "(split the batch)", (unsigned long long)n, (unsigned long long)need,
                    (unsigned long long)kStaticScratchBytes);
    if (n == 0) return PS_OK;
    char* base = nullptr;
    rc = scratch_for_current_device(&base);
    if (rc != PS_OK) return rc;
    Work w;
    DevSpectra dsp;
    layout_work(n, nnz, kp, false, items, base, &w, nullptr, 0);
    w.hits = hits;                        // results go straight to the caller's buffers
    w.stats = stats;
    if (hist) w.hist = hist;
    dsp.peak_off = spectra->peak_off;
    dsp.mz = spectra->mz;
    dsp.inten = spectra->intensity;
    dsp.prec = spectra->precursor_mz;
    dsp.charge = spectra->charge;
    dsp.n = n;
    dsp.nnz = nnz;
    dsp.hdr = w.hdr;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = launch_set_header(w.hdr, n, nnz, st);
    if (e == hipSuccess) e = enqueue_kernels(ix, dsp, kp, sc, params->schedule, w, false, st, nullptr, nullptr);
    if (e != hipSuccess) return fail(PS_EDEVICE, "static search: %s", hipGetErrorString(e));
    return PS_OK;
}

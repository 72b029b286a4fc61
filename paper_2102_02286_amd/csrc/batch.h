// batch.h -- the object behind a ps_batch handle and the launch schedule.
#pragma once
#include "state.h"

namespace ps {

using Schedule = ps_schedule;
Schedule default_schedule();
int make_kparams(const ps_index* ix, const ps_search_params* p, KParams* kp, const Schedule* sched);
int check_schedule(const Schedule& s);
hipError_t enqueue_kernels(const ps_index* ix, const DevSpectra& dsp, const KParams& kp, const Schedule& sc,
                           int schedule, const Work& w, bool dump, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
uint64_t layout_work(uint64_t n, uint64_t nnz, const KParams& kp, bool copy_inputs, uint64_t max_items,
                     char* base, Work* w, DevSpectra* dsp, uint64_t dump_cap);
uint64_t max_items_for(const ps_index* ix, uint64_t n, const KParams& kp, const Schedule& sc, int schedule);
int validate_host_spectra(const ps_spectra* sp, const KParams& kp);

}  // namespace ps

struct ps_batch {
    ps_index* ix = nullptr;
    uint64_t n = 0;
    ps::KParams kp{};
    ps::Schedule sched{};
    int schedule = PS_SCHED_PLAIN;
    bool want_hist = false;
    bool dump = false;
    hipStream_t stream = nullptr;
    uint64_t max_items = 0;
    uint32_t grid = 0;
    uint32_t scan_launches = 0;
    ps::Work w{};
    ps::DevSpectra dsp{};
    hipEvent_t ev_scan0 = nullptr, ev_scan1 = nullptr, ev_done = nullptr;
    ps_hit* h_hits = nullptr;
    ps_stat* h_stats = nullptr;
    int32_t* h_hist = nullptr;
    unsigned long long* h_counters = nullptr;
    char* h_stage = nullptr;
    ps::BatchHdr* h_hdr = nullptr;
};

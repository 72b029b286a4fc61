// batch.h -- the object behind a ps_batch handle and the launch schedule.
#pragma once
#include "state.h"

namespace ps {

using Schedule = ps_schedule;
Schedule default_schedule();
int make_kparams(const ps_index* ix, const ps_search_params* p, KParams* kp, const Schedule* sched);

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
};

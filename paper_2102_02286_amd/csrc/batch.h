// batch.h -- the object behind a ps_batch handle and the launch schedule.
#pragma once
#include "state.h"

namespace ps {

// Launch shape of the scan (chosen by default or by the autotuner).
struct Schedule {
    uint32_t tile;            // candidates per LDS counter tile
    uint32_t heavy_min;       // segments longer than this are streamed by the whole workgroup
    uint32_t tiles_per_item;  // persistent schedule: tiles per work item
    uint32_t grid_per_cu;     // persistent schedule: workgroups per compute unit
};

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

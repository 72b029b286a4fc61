// autotune.cpp -- pick the scan schedule by measurement.
//
// Coordinate descent over the schedule fields (tile, and for the persistent
// schedule the work-item size and resident workgroups per CU): each candidate searches a sample batch, its
// scan is timed with HIP events, and its results must equal the baseline's
// bit for bit (a schedule only changes speed).  The winner is set on the index
// and, if a cache file is given, stored under a key made of the index shape
// and the search parameters, so later processes skip the search.
#include "batch.h"

#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

using namespace ps;

extern "C" {
int ps_search_batch(ps_index* idx, const ps_device* work, const ps_spectra* spectra, const ps_search_params* params,
                    ps_batch** out);
int ps_results(ps_batch* batch, ps_hit* hits, ps_stat* stats, int32_t* hist);
int ps_batch_timing(ps_batch* batch, double* scan_ms, uint32_t* scan_launches, uint64_t* postings,
                    uint64_t* bin_lookups);
void ps_batch_free(ps_batch* batch);
int ps_workspace_bytes(const ps_index* idx, uint64_t n, uint64_t nnz, const ps_search_params* params,
                       uint64_t* bytes);
}

namespace {

std::string cache_key(const ps_index* ix, const ps_search_params* p) {
    std::ostringstream k;
    k << "D" << ix->n_entries << "_N" << n_postings(ix) << "_ppm" << p->window_is_ppm << "_w" << p->window
      << "_T" << p->frag_tol_bins << "_B" << p->top_peaks << "_k" << p->top_k << "_z" << p->max_charge << "_s"
      << p->schedule;
    return k.str();
}

bool cache_lookup(const char* path, const std::string& key, ps_schedule* out) {
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        ps_schedule s{};
        if (is >> k >> s.tile >> s.tiles_per_item >> s.groups_per_cu >> s.group_threads && k == key) {
            *out = s;
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& key, const ps_schedule& s) {
    if (!path) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line)) {
            std::istringstream is(line);
            std::string k;
            if (is >> k && k != key) keep.push_back(line);
        }
    }
    std::ofstream f(path, std::ios::trunc);
    for (auto& l : keep) f << l << "\n";
    f << key << " " << s.tile << " " << s.tiles_per_item << " " << s.groups_per_cu << " " << s.group_threads
      << "\n";
}

struct Outcome {
    int rc = PS_OK;
    double ms = 0;
    std::vector<ps_hit> hits;
    std::vector<ps_stat> stats;
};

Outcome run_once(ps_index* ix, const ps_device* work, const ps_spectra* sp, const ps_search_params* p) {
    Outcome o;
    uint64_t need = 0;
    const uint64_t nnz = sp->n ? sp->peak_off[sp->n] : 0;
    o.rc = ps_workspace_bytes(ix, sp->n, nnz, p, &need);
    if (o.rc != PS_OK) return o;
    if (need > work->bytes) { o.rc = PS_ENOMEM; return o; }
    ps_batch* b = nullptr;
    o.rc = ps_search_batch(ix, work, sp, p, &b);
    if (o.rc != PS_OK) return o;
    o.hits.resize(sp->n * p->top_k);
    o.stats.resize(sp->n);
    o.rc = ps_results(b, o.hits.data(), o.stats.data(), nullptr);
    if (o.rc == PS_EOVERFLOW) o.rc = PS_OK;
    if (o.rc == PS_OK) o.rc = ps_batch_timing(b, &o.ms, nullptr, nullptr, nullptr);
    ps_batch_free(b);
    return o;
}

bool same(const Outcome& a, const Outcome& b) {
    return a.hits.size() == b.hits.size() && a.stats.size() == b.stats.size() &&
           memcmp(a.hits.data(), b.hits.data(), a.hits.size() * sizeof(ps_hit)) == 0 &&
           memcmp(a.stats.data(), b.stats.data(), a.stats.size() * sizeof(ps_stat)) == 0;
}

}  // namespace

extern "C" int ps_autotune(ps_index* ix, const ps_device* work, const ps_spectra* sample,
                           const ps_search_params* params, const char* cache_path, ps_tune_trial* trials,
                           uint32_t max_trials, uint32_t* n_trials, ps_schedule* best) {
    if (!ix || !work || !sample || !params) return fail(PS_EINVAL, "NULL argument");
    if (n_trials) *n_trials = 0;
    const std::string key = cache_key(ix, params);
    ps_schedule cached;
    if (cache_lookup(cache_path, key, &cached) && check_schedule(cached) == PS_OK) {
        ix->sched = cached;
        if (best) *best = cached;
        return PS_OK;
    }
    const ps_schedule start = ix->sched;
    uint32_t nt = 0;
    auto record = [&](const ps_schedule& s, double ms, bool ok) {
        if (trials && nt < max_trials) { trials[nt].schedule = s; trials[nt].scan_ms = ms; trials[nt].same = ok; }
        ++nt;
    };
    auto measure = [&](const ps_schedule& s, Outcome* ref, double* ms_out) -> int {
        ix->sched = s;
        Outcome warm = run_once(ix, work, sample, params);         // first run: code and caches warm
        if (warm.rc != PS_OK) return warm.rc;
        Outcome o = run_once(ix, work, sample, params);
        if (o.rc != PS_OK) return o.rc;
        const bool ok = ref ? same(o, *ref) : true;
        record(s, o.ms, ok);
        if (!ok) return fail(PS_EDEVICE, "schedule (tile %u) changed the results", s.tile);
        *ms_out = o.ms;
        return PS_OK;
    };
    Outcome ref = run_once(ix, work, sample, params);
    if (ref.rc != PS_OK) { ix->sched = start; return ref.rc; }
    ps_schedule cur = start;
    double cur_ms = 0;
    int rc = measure(cur, &ref, &cur_ms);
    if (rc != PS_OK) { ix->sched = start; return rc; }
    const bool persistent = params->schedule == PS_SCHED_PERSISTENT;
    for (int pass = 0; pass < 2; ++pass) {
        bool improved = false;
        for (int field = 0; field < 3; ++field) {
            // field 0: (threads per workgroup, tile) pairs, coded as threads << 16 | tile / 1024
            std::vector<uint32_t> vals;
            switch (field) {
                case 0: vals = {256u << 16 | 4, 256u << 16 | 8, 256u << 16 | 16, 512u << 16 | 8, 512u << 16 | 16};
                        break;
                case 1: if (persistent) vals = {8, 16, 32, 64, 128, 256}; break;
                case 2: if (persistent) vals = {3, 4, 5, 6, 8}; break;
            }
            for (uint32_t v : vals) {
                ps_schedule s = cur;
                if (field == 0) {
                    const uint32_t gt = v >> 16, tile = (v & 0xFFFFu) * 1024u;
                    if (s.tile == tile && (s.group_threads ? s.group_threads : 256u) == gt) continue;
                    s.tile = tile;
                    s.group_threads = gt;
                } else {
                    uint32_t* f = field == 1 ? &s.tiles_per_item : &s.groups_per_cu;
                    if (*f == v) continue;
                    *f = v;
                }
                if (check_schedule(s) != PS_OK || s.tile < (1u << ix->dir_shift)) continue;
                double ms = 0;
                rc = measure(s, &ref, &ms);
                if (rc == PS_ENOMEM || rc == PS_EINVAL) continue;   // does not fit this block / LDS
                if (rc != PS_OK) { ix->sched = start; return rc; }
                if (ms < cur_ms * 0.98) { cur = s; cur_ms = ms; improved = true; }
            }
        }
        if (!improved) break;
    }
    ix->sched = cur;
    if (best) *best = cur;
    if (n_trials) *n_trials = nt;
    cache_store(cache_path, key, cur);
    return PS_OK;
}

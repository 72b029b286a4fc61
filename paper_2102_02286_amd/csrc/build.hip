// build.hip -- the fragment-ion index built on the device.
//
// Superstep 1 of HiCOPS (arXiv 2102.02286; Supplementary Algorithm 1): generate
// every database entry, sort the entries, generate their b/y ions and index
// them.  The same index as index_build_host, bit for bit, made on the GPU:
//   1. host: count the entries (peptides x modification subsets) of every
//      cleavage start with binomial sums, which fixes where each start's entries
//      go (no materialisation on the host);
//   2. k_gen_entries: one thread per start writes its entries in (length, site
//      mask) order; starts are in (protein, position) order, so generation order
//      is the tie order of the key (mass, protein, start, length, mask);
//   3. a stable radix sort by mass then gives the id order; a partition keeps
//      every G-th rank;
//   4. ions: per entry 2(n-1) b/y ions, each posted to the 2T+1 bins of a
//      merged list (T = 0: one bin).  In chunks of entries the (bin, posting)
//      pairs are generated in id order and stably sorted by bin.  A first pass
//      adds each chunk's per-bin run lengths; the host turns the counts into
//      list offsets, each list padded to whole 16-byte quads; a second pass
//      scatters every chunk's runs behind each bin's cursor (a single chunk
//      stays sorted between the passes) -- a chunked counting sort, so every
//      list is in id order and the scratch memory is bounded by the chunk;
//   5. k_dir: the tile directory, one binary search per (bin, block), as
//      positions inside the bin's list.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "batch.h"
#include "state.h"

namespace ps {

namespace {

constexpr uint64_t kChunkPairs = 1ull << 29;   // (bin, posting) pairs sorted at a time (8.6 GB of buffers)

__constant__ int64_t c_residue[26] = {
    71037114, -1, 103009185, 115026943, 129042593, 147068414, 57021464, 137058912,   // A..H
    113084064, -1, 128094963, 113084064, 131040485, 114042927, -1, 97052764,         // I..P
    128058578, 156101111, 87032028, 101047679, -1, 99068414, 186079313, -1,          // Q..X
    163063329, -1,                                                                     // Y, Z
};

struct ModArgs {
    int32_t res_mod[26];
    int32_t nterm_mod;
    int32_t pad;
    int64_t delta[16];
};

__device__ __forceinline__ bool cut_after(const char* s, uint64_t n, uint64_t i) {
    if (s[i] != 'K' && s[i] != 'R') return false;
    return i + 1 >= n || s[i + 1] != 'P';
}

// Mass shift of the modification sites selected by `mask` (bit order: the
// protein N-terminus first when the peptide starts the protein, then residues by
// position).
__device__ int64_t site_shift(const char* s, uint32_t a, uint32_t len, uint64_t mask, const ModArgs& M) {
    int64_t d = 0;
    uint32_t bit = 0;
    if (a == 0 && M.nterm_mod >= 0) {
        if (mask & 1ull) d += M.delta[M.nterm_mod];
        bit = 1;
    }
    for (uint32_t j = 0; j < len; ++j) {
        const int mm = M.res_mod[s[a + j] - 'A'];
        if (mm >= 0) {
            if (mask >> bit & 1ull) d += M.delta[mm];
            ++bit;
        }
    }
    return d;
}

struct GenArgs {
    const char* seq;
    const uint64_t* prot_off;
    const uint32_t* st_prot;     // cleavage starts with entries: protein, position, first entry
    const uint32_t* st_pos;
    const uint64_t* st_off;
    uint64_t n_starts;
    uint32_t missed, min_len, max_len, max_mods;
    ModArgs mods;
    int64_t min_mass;
    int64_t* mass;
    uint32_t* prot;
    uint32_t* start;
    uint8_t* len;
    uint64_t* mask;
    uint64_t* key;               // mass - min_mass, the sort key
    uint32_t* idx;               // generation index, the sort payload
};

// One thread per cleavage start: every peptide from it (trypsin, missed
// cleavages, length range), and for each every subset of <= max_mods sites in
// increasing mask order.  The walk is the host census's walk, so entry k of
// start i lands at st_off[i] + k.
__global__ void k_gen_entries(GenArgs A) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < A.n_starts;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = A.st_prot[i];
        const uint64_t a = A.st_pos[i];
        const char* s = A.seq + A.prot_off[p];
        const uint64_t n = A.prot_off[p + 1] - A.prot_off[p];
        uint64_t o = A.st_off[i];
        uint32_t missed = 0;
        int64_t base = kWaterUda;
        for (uint64_t e = a + 1; e <= n; ++e) {
            const uint64_t len = e - a;
            if (len > A.max_len) break;
            base += c_residue[s[e - 1] - 'A'];
            const bool end = (e == n) || cut_after(s, n, e - 1);
            if (!end) continue;
            if (len >= A.min_len) {
                uint32_t ns = (a == 0 && A.mods.nterm_mod >= 0) ? 1u : 0u;
                for (uint64_t j = a; j < e; ++j) ns += A.mods.res_mod[s[j] - 'A'] >= 0 ? 1u : 0u;
                const uint64_t full = ns >= 64 ? ~0ull : (1ull << ns) - 1ull;   // ns <= 63 (checked)
                uint64_t mask = 0;
                while (true) {
                    const int64_t m = base + site_shift(s, (uint32_t)a, (uint32_t)len, mask, A.mods);
                    A.mass[o] = m;
                    A.prot[o] = p;
                    A.start[o] = (uint32_t)a;
                    A.len[o] = (uint8_t)len;
                    A.mask[o] = mask;
                    A.key[o] = (uint64_t)(m - A.min_mass);
                    A.idx[o] = (uint32_t)o;
                    ++o;
                    // next mask in increasing order with at most max_mods bits: a mask with
                    // too many bits is skipped together with every mask that only adds
                    // bits below its lowest one
                    uint64_t y = mask + 1;
                    while (y != 0 && y <= full && (uint32_t)__popcll(y) > A.max_mods) y += y & (~y + 1);
                    if (y == 0 || y > full) break;
                    mask = y;
                }
            }
            if (e < n && ++missed > A.missed) break;
        }
    }
}

struct TakeArgs {
    const uint32_t* order;       // generation index of each sorted rank
    uint64_t n_local, G, g;
    const int64_t* mass_in;
    const uint32_t* prot_in;
    const uint32_t* start_in;
    const uint8_t* len_in;
    const uint64_t* mask_in;
    int64_t* mass;               // index block
    uint32_t* prot;
    uint32_t* start;
    uint8_t* len;
    uint64_t* mask;
    uint64_t* pair_cnt;          // [n_local + 1] pairs of each entry (last = 0)
    uint32_t pairs_per_ion;      // (2T + 1) x enabled ion series
};

// Ranks r * G + g of the sorted database become this partition's ids r.
__global__ void k_take(TakeArgs A) {
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r <= A.n_local;
         r += (uint64_t)gridDim.x * blockDim.x) {
        if (r == A.n_local) { A.pair_cnt[r] = 0; continue; }
        const uint32_t src = A.order[r * A.G + A.g];
        A.mass[r] = A.mass_in[src];
        A.prot[r] = A.prot_in[src];
        A.start[r] = A.start_in[src];
        A.len[r] = A.len_in[src];
        A.mask[r] = A.mask_in[src];
        A.pair_cnt[r] = (uint64_t)(A.len_in[src] - 1) * A.pairs_per_ion;
    }
}

struct IonArgs {
    const char* seq;
    const uint64_t* prot_off;
    const uint32_t* prot;
    const uint32_t* start;
    const uint8_t* len;
    const uint64_t* mask;
    ModArgs mods;
    IonSeries ions;              // enabled series, N-terminal first
    int32_t T;                   // merge width (0: classic lists)
    uint64_t n_bins;
    uint64_t r0, r1;             // entries of this pass
    const uint64_t* pair_off;    // [n + 1] first pair of each entry
    uint32_t* key;               // bin, posting (chunk-relative positions)
    uint32_t* val;
    int* bad;                    // set when an ion has a negative mass or leaves the bin range
};

// Residue j of an entry with its modification folded in (the N-terminal shift
// goes to residue 0).  `bit` is the site counter, advanced past residue j.
__device__ __forceinline__ int64_t residue_at(const char* s, uint32_t j, uint64_t mask, uint32_t& bit,
                                              const ModArgs& M) {
    int64_t m = c_residue[s[j] - 'A'];
    const int mm = M.res_mod[s[j] - 'A'];
    if (mm >= 0) {
        if (mask >> bit & 1ull) m += M.delta[mm];
        ++bit;
    }
    return m;
}

// One thread per entry: for every enabled series, N-terminal ones first, the
// ions i = 1..n-1 (residues 1..i, or n-i+1..n for C-terminal series), each to
// bins bin-T..bin+T, written as (bin, posting) pairs in this order, so a stable
// sort by bin keeps every list in (id, N-terminal before C-terminal) order.
__global__ void k_ions(IonArgs A) {
    for (uint64_t r = A.r0 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < A.r1;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const char* s = A.seq + A.prot_off[A.prot[r]] + A.start[r];
        const uint32_t n = A.len[r];
        const uint64_t mask = A.mask[r];
        const bool nt = A.start[r] == 0 && A.mods.nterm_mod >= 0;
        const int64_t nshift = (nt && (mask & 1ull)) ? A.mods.delta[A.mods.nterm_mod] : 0;
        uint32_t nsites = nt ? 1u : 0u;                  // every site, for the backward walks
        for (uint32_t j = 0; j < n; ++j) nsites += A.mods.res_mod[s[j] - 'A'] >= 0 ? 1u : 0u;
        uint64_t w = A.pair_off[r] - A.pair_off[A.r0];
        for (int t = 0; t < A.ions.n; ++t) {
            const bool y = A.ions.cterm[t] != 0;
            uint32_t bit = nt ? 1u : 0u;
            uint32_t bit_back = nsites;
            int64_t acc = 0;
            for (uint32_t i = 1; i < n; ++i) {
                int64_t ion;
                if (!y) {
                    acc += residue_at(s, i - 1, mask, bit, A.mods) + (i == 1 ? nshift : 0);
                    ion = acc + kProtonUda + A.ions.shift[t];
                } else {
                    // residue n-i: its site bit is the number of sites before it
                    const uint32_t j = n - i;
                    const int mm = A.mods.res_mod[s[j] - 'A'];
                    if (mm >= 0) --bit_back;
                    int64_t m = c_residue[s[j] - 'A'];
                    if (mm >= 0 && (mask >> bit_back & 1ull)) m += A.mods.delta[mm];
                    acc += m;
                    ion = acc + kWaterUda + kProtonUda + A.ions.shift[t];
                }
                if (ion < 0) { atomicOr(A.bad, 1); continue; }
                const int64_t bn = (ion + kBinWidth / 2) / kBinWidth;
                for (int d = -A.T; d <= A.T; ++d) {
                    const int64_t b2 = bn + d;
                    if (b2 < 0 || b2 >= (int64_t)A.n_bins) { atomicOr(A.bad, 2); continue; }
                    A.key[w] = (uint32_t)b2;
                    A.val[w] = (uint32_t)(r << 1) | (uint32_t)y;
                    ++w;
                }
            }
        }
    }
}

struct ScatterArgs {
    const uint32_t* key;         // sorted chunk
    const uint32_t* val;
    uint64_t m;
    uint32_t* run_start;         // [n_bins] first position of each bin's run in the chunk
    uint32_t* run_end;
    const uint32_t* bin_q;       // [n_bins] first quad of each bin's list
    unsigned long long* cursor;  // [n_bins] postings of the bin written so far
    uint32_t* post;
};

__global__ void k_runs(ScatterArgs A) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < A.m; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t b = A.key[i];
        if (i == 0 || A.key[i - 1] != b) A.run_start[b] = (uint32_t)i;
        if (i + 1 == A.m || A.key[i + 1] != b) A.run_end[b] = (uint32_t)(i + 1);
    }
}

__global__ void k_scatter(ScatterArgs A) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < A.m; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t b = A.key[i];
        A.post[4ull * A.bin_q[b] + A.cursor[b] + (i - A.run_start[b])] = A.val[i];
    }
}

__global__ void k_advance(ScatterArgs A) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < A.m; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t b = A.key[i];
        if (i == 0 || A.key[i - 1] != b) A.cursor[b] += A.run_end[b] - A.run_start[b];
    }
}

// Postings of each bin in a sorted chunk: cnt[b] += (first position > b) -
// (first position >= b), by binary search, for b < n_bins.
__global__ void k_bin_runs(const uint32_t* key, uint64_t m, uint64_t n_bins, unsigned long long* cnt) {
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < n_bins;
         b += (uint64_t)gridDim.x * blockDim.x) {
        auto first_ge = [&](uint64_t v) {
            uint64_t lo = 0, hi = m;
            while (lo < hi) {
                const uint64_t mid = (lo + hi) >> 1;
                if ((uint64_t)key[mid] < v) lo = mid + 1; else hi = mid;
            }
            return lo;
        };
        cnt[b] += first_ge(b + 1) - first_ge(b);
    }
}

__global__ void k_fill_post(uint32_t* p, uint32_t v, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_u64(unsigned long long* p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Entry k of bin b: the position in b's list of its first posting with id >=
// k << shift.
__global__ void k_dir(const uint32_t* bin_q, const unsigned long long* bin_cnt, const uint32_t* post, uint64_t n_bins,
                      uint64_t stride, uint32_t shift, uint32_t* dir) {
    const uint64_t total = n_bins * stride;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t b = t / stride, k = t - b * stride;
        const uint64_t target = (k << shift) << 1;          // posting = id << 1 | y
        const uint32_t* list = post + 4ull * bin_q[b];
        uint64_t lo = 0, hi = bin_cnt[b];
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if ((uint64_t)list[mid] < target) lo = mid + 1; else hi = mid;
        }
        dir[t] = (uint32_t)lo;
    }
}

uint32_t grid_for(uint64_t n, uint32_t block = 256) {
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (uint32_t)g;
}

uint32_t bit_length(uint64_t x) { return x ? 64u - (uint32_t)__builtin_clzll(x) : 1u; }

// Host count: entries per protein and the quantities the layout needs.
struct Census {
    std::vector<uint32_t> st_prot, st_pos;   // cleavage starts with at least one entry
    std::vector<uint64_t> st_off;            // [starts + 1] first entry of each start
    uint64_t D_all = 0;
    int64_t min_mass = 0, max_mass = 0;
    uint32_t max_len = 0;
    uint64_t D = 0, n_bins = 0, post_cap = 0, quad_cap = 0, dir_stride = 0, dir_nblk = 0;
    uint32_t dir_shift = 12;
};

int census(const ps_index* ix, Census& C) {
    const ModTable mt = mod_table(ix);
    const uint64_t n_prot = ix->prot_off.size() - 1;
    const uint32_t series = (uint32_t)__builtin_popcount(ix->ion_types);
    uint64_t binom[64][64];
    for (int a = 0; a < 64; ++a)
        for (int b = 0; b < 64; ++b) binom[a][b] = b == 0 ? 1 : (a == 0 ? 0 : binom[a - 1][b - 1] + binom[a - 1][b]);
    const unsigned T = worker_threads();
    struct Part {
        int64_t lo = INT64_MAX, hi = INT64_MIN; uint32_t max_len = 0; uint64_t pairs = 0;
        std::vector<uint32_t> prot, pos; std::vector<uint64_t> cnt;
    };
    std::vector<Part> parts(T);
    std::atomic<int> bad{0};
    const uint64_t chunk = (n_prot + T - 1) / std::max<uint64_t>(T, 1);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; ++t) {
        const uint64_t pa = t * chunk, pb = std::min(n_prot, pa + chunk);
        if (pa >= pb) break;
        th.emplace_back([&, t, pa, pb] {
            Part& P = parts[t];
            int64_t site[64];
            for (uint64_t p = pa; p < pb; ++p) {
                const char* s = ix->seq.data() + ix->prot_off[p];
                const uint64_t n = ix->prot_off[p + 1] - ix->prot_off[p];
                for (uint64_t a = 0; a < n; ++a) {
                    if (a != 0 && !is_cut(s, n, a - 1)) continue;
                    uint64_t c = 0;
                    uint32_t missed = 0;
                    int64_t base = kWaterUda;
                    for (uint64_t e = a + 1; e <= n; ++e) {
                        const uint64_t len = e - a;
                        if (len > ix->max_len) break;
                        base += residue_uda(s[e - 1]);
                        const bool end = (e == n) || is_cut(s, n, e - 1);
                        if (!end) continue;
                        if (len >= ix->min_len) {
                            uint32_t ns = 0;
                            if (a == 0 && mt.nterm_mod >= 0) site[ns++] = ix->mods[mt.nterm_mod].delta;
                            for (uint64_t j = a; j < e && ns <= 63; ++j) {
                                const int mm = mt.res_mod[s[j] - 'A'];
                                if (mm >= 0) site[ns++] = ix->mods[mm].delta;
                            }
                            if (ns > 63) { bad = 1; continue; }
                            const uint32_t k = std::min<uint32_t>(ix->max_mods, ns);
                            uint64_t v = 0;
                            for (uint32_t i = 0; i <= k; ++i) v += binom[ns][i];
                            if (v >= (1ull << 31)) { bad = 2; continue; }
                            c += v;
                            // lightest and heaviest variant: the k most negative / positive shifts
                            std::sort(site, site + ns);
                            int64_t lo = base, hi = base;
                            for (uint32_t i = 0; i < k && site[i] < 0; ++i) lo += site[i];
                            for (uint32_t i = 0; i < k && site[ns - 1 - i] > 0; ++i) hi += site[ns - 1 - i];
                            P.lo = std::min(P.lo, lo);
                            P.hi = std::max(P.hi, hi);
                            P.max_len = std::max(P.max_len, (uint32_t)len);
                            P.pairs += v * (uint64_t)series * (len - 1);
                        }
                        if (e < n && ++missed > ix->missed) break;
                    }
                    if (c) { P.prot.push_back((uint32_t)p); P.pos.push_back((uint32_t)a); P.cnt.push_back(c); }
                }
            }
        });
    }
    for (auto& x : th) x.join();
    if (bad == 1) return fail(PS_EINVAL, "a peptide has more than 63 modifiable sites");
    if (bad == 2) return fail(PS_EOVERFLOW, "one peptide has 2^31 or more modified forms");
    C.st_off.assign(1, 0);
    for (Part& P : parts) {                   // threads hold consecutive protein ranges
        C.st_prot.insert(C.st_prot.end(), P.prot.begin(), P.prot.end());
        C.st_pos.insert(C.st_pos.end(), P.pos.begin(), P.pos.end());
        for (uint64_t c : P.cnt) {
            C.st_off.push_back(C.st_off.back() + c);
            if (C.st_off.back() >= (1ull << 31)) return fail(PS_EOVERFLOW, "more than 2^31 database entries");
        }
        std::vector<uint32_t>().swap(P.prot); std::vector<uint32_t>().swap(P.pos); std::vector<uint64_t>().swap(P.cnt);
    }
    C.D_all = C.st_off.back();
    C.min_mass = INT64_MAX;
    C.max_mass = INT64_MIN;
    uint64_t pairs_all = 0;
    for (const Part& P : parts) {
        C.min_mass = std::min(C.min_mass, P.lo);
        C.max_mass = std::max(C.max_mass, P.hi);
        C.max_len = std::max(C.max_len, P.max_len);
        pairs_all += P.pairs;
    }
    if (C.D_all == 0) { C.min_mass = 0; C.max_mass = 0; }
    const uint64_t G = ix->n_shards, g = ix->shard;
    C.D = C.D_all > g ? (C.D_all - g + G - 1) / G : 0;
    C.n_bins = (uint64_t)((std::max<int64_t>(C.max_mass, 0) + kBinWidth / 2) / kBinWidth) + 2;
    if (C.n_bins >= (1ull << 24))
        return fail(PS_EOVERFLOW, "peptide masses need %llu fragment bins (limit 2^24)", (unsigned long long)C.n_bins);
    const uint64_t width = 2ull * ix->merge_tol + 1;
    // postings: exact for the whole database; a partition's share is bounded by
    // its entry count times the longest peptide's ions
    uint64_t cap = pairs_all * width;
    if (G > 1) cap = std::min<uint64_t>(cap, C.D * (uint64_t)series * (C.max_len > 0 ? C.max_len - 1 : 0) * width);
    C.post_cap = cap;
    C.quad_cap = (cap + 3) / 4 + C.n_bins;   // every list padded to whole quads
    C.dir_shift = directory_shift(C.n_bins, C.D);
    C.dir_nblk = (C.D >> C.dir_shift) + 1;
    C.dir_stride = (C.dir_nblk + 1 + 3) & ~3ull;
    return PS_OK;
}

uint64_t a256(uint64_t x) { return (x + 255) & ~255ull; }

// Scratch layout of a build; sizes only when base is NULL.
struct Scratch {
    char* seq; uint64_t* prot_off; uint32_t* st_prot; uint32_t* st_pos; uint64_t* st_off;
    int64_t* g_mass; uint32_t* g_prot; uint32_t* g_start; uint8_t* g_len; uint64_t* g_mask;
    uint64_t* key0; uint64_t* key1; uint32_t* idx0; uint32_t* idx1;
    uint32_t* l_prot; uint32_t* l_start; uint8_t* l_len; uint64_t* l_mask;   // in the index block
    uint64_t* pair_cnt; uint64_t* pair_off;
    unsigned long long* bin_cnt; uint32_t* bin_q; unsigned long long* cursor; uint32_t* run_start; uint32_t* run_end;
    uint32_t* pk0; uint32_t* pk1; uint32_t* pv0; uint32_t* pv1;
    int* bad;
    void* temp; uint64_t temp_bytes;
    uint64_t total;
};

Scratch layout_scratch(char* base, const ps_index* ix, const Census& C, uint64_t chunk, uint64_t temp_bytes) {
    Scratch S{};
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) { uint64_t at = o; o = a256(o + bytes); return base ? base + at : nullptr; };
    const uint64_t np = ix->prot_off.size();
    const uint64_t Da = std::max<uint64_t>(C.D_all, 1), D = std::max<uint64_t>(C.D, 1);
    S.seq = (char*)take(ix->seq.size() + 1);
    S.prot_off = (uint64_t*)take(np * 8);
    const uint64_t ns = std::max<uint64_t>(C.st_prot.size(), 1);
    S.st_prot = (uint32_t*)take(ns * 4);
    S.st_pos = (uint32_t*)take(ns * 4);
    S.st_off = (uint64_t*)take((ns + 1) * 8);
    S.g_mass = (int64_t*)take(Da * 8);
    S.g_prot = (uint32_t*)take(Da * 4);
    S.g_start = (uint32_t*)take(Da * 4);
    S.g_len = (uint8_t*)take(Da);
    S.g_mask = (uint64_t*)take(Da * 8);
    S.key0 = (uint64_t*)take(Da * 8);
    S.key1 = (uint64_t*)take(Da * 8);
    S.idx0 = (uint32_t*)take(Da * 4);
    S.idx1 = (uint32_t*)take(Da * 4);
    S.pair_cnt = (uint64_t*)take((D + 1) * 8);
    S.pair_off = (uint64_t*)take((D + 1) * 8);
    S.bin_cnt = (unsigned long long*)take((C.n_bins + 1) * 8);
    S.bin_q = (uint32_t*)take((C.n_bins + 1) * 4);
    S.cursor = (unsigned long long*)take(C.n_bins * 8);
    S.run_start = (uint32_t*)take(C.n_bins * 4);
    S.run_end = (uint32_t*)take(C.n_bins * 4);
    S.pk0 = (uint32_t*)take(chunk * 4);
    S.pk1 = (uint32_t*)take(chunk * 4);
    S.pv0 = (uint32_t*)take(chunk * 4);
    S.pv1 = (uint32_t*)take(chunk * 4);
    S.bad = (int*)take(256);
    S.temp = take(temp_bytes);
    S.temp_bytes = temp_bytes;
    S.total = o;
    return S;
}

// Workspace of the library sorts and scans at these sizes (no launch).
uint64_t temp_bytes_for(const Census& C, uint64_t chunk, hipStream_t st, hipError_t* err) {
    size_t a = 0, b = 0, c = 0;
    hipcub::DoubleBuffer<uint64_t> k64(nullptr, nullptr);
    hipcub::DoubleBuffer<uint32_t> v32(nullptr, nullptr);
    hipcub::DoubleBuffer<uint32_t> k32(nullptr, nullptr);
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, a, k64, v32, (int)std::max<uint64_t>(C.D_all, 1), 0,
                                                      64, st);
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(nullptr, b, k32, v32, (int)std::max<uint64_t>(chunk, 1), 0, 32, st);
    if (e == hipSuccess)
        e = hipcub::DeviceScan::ExclusiveSum(nullptr, c, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                             (int)(std::max<uint64_t>(C.D, 1) + 1), st);
    *err = e;
    return std::max(std::max(a, b), c) + 4096;
}

// Pairs per chunk: the caller's cap (0: the default), at least one entry's
// worth, at most what the database has.
uint64_t chunk_pairs(const Census& C, uint64_t cap, uint32_t width) {
    const uint64_t one = 6ull * (C.max_len > 0 ? C.max_len - 1 : 0) * width;   // six series at most
    uint64_t c = cap ? cap : kChunkPairs;
    c = std::max<uint64_t>(c, one);
    return std::max<uint64_t>(1, std::min<uint64_t>(C.post_cap, c));
}

}  // namespace

}  // namespace ps

using namespace ps;

// One list's dense map: every posting sets its id's bit (C-terminal bits
// 0-3, N-terminal bits 4-7 of byte id / 4).  flags bit 0: a bit was already
// set (the list repeats an (id, terminus) pair, which a map cannot hold);
// bit 1: some id has postings of both termini (a probe on the list can add 2
// to that id's count).
// Grid-stride: a list can hold more postings than one capped grid has threads.
__global__ void k_dense_map(const uint32_t* list, uint64_t len, uint32_t* map, uint32_t* flags) {
    const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    uint32_t f = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += step) {
        const uint32_t p = list[i];
        const uint32_t id = p >> 1;
        const uint32_t bit = ((id >> 2) & 3u) * 8u + (id & 3u) + ((p & 1u) ? 0u : 4u);
        const uint32_t old = atomicOr(&map[id >> 4], 1u << bit);
        if (old & (1u << bit)) f |= 1u;
        if (old & (1u << (bit ^ 4u))) f |= 2u;
    }
    if (f) atomicOr(flags, f);
}

namespace ps {

int build_dense_maps(ps_index* ix, char* base, const DevLayout& lay, hipStream_t st) {
    ix->n_dense = 0;
    bind_dense(ix);
    const std::vector<uint32_t> cand = dense_candidates(ix);
    const uint32_t nc = std::min<uint32_t>((uint32_t)cand.size(), lay.dense_cap);
    if (nc == 0) return PS_OK;
    // first quad of every bin's padded list
    std::vector<uint64_t> q0(ix->n_bins + 1, 0);
    for (uint64_t b = 0; b < ix->n_bins; ++b) q0[b + 1] = q0[b] + ((ix->bin_off[b + 1] - ix->bin_off[b] + 3) >> 2);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    uint32_t* flags = (uint32_t*)(base + lay.dense_flags);
    chk(launch_fill_u32(base + lay.dense, 0u, (uint64_t)nc * lay.dense_stride / 4, st));
    chk(launch_fill_u32(flags, 0u, kMaxDense, st));
    for (uint32_t k = 0; k < nc && e == hipSuccess; ++k) {
        const uint32_t b = cand[k];
        const uint64_t len = ix->bin_off[b + 1] - ix->bin_off[b];
        hipLaunchKernelGGL(k_dense_map, dim3(grid_for(len)), dim3(256), 0, st, ix->dev.post + 4 * q0[b], len,
                           (uint32_t*)(base + lay.dense + (uint64_t)k * lay.dense_stride), flags + k);
        chk(hipGetLastError());
    }
    uint32_t rep[kMaxDense] = {};
    chk(hipMemcpyAsync(rep, flags, sizeof rep, hipMemcpyDeviceToHost, st));
    chk(hipStreamSynchronize(st));
    if (e != hipSuccess) return fail(PS_EDEVICE, "dense maps: %s", hipGetErrorString(e));
    uint32_t tab[kMaxDense] = {};
    uint32_t n = 0;
    for (uint32_t k = 0; k < nc; ++k) {
        if ((rep[k] & 1u) || cand[k] >= (1u << 24)) continue;   // the list stays postings only
        ix->dense_bin[n] = cand[k];
        tab[n] = cand[k] | ((rep[k] & 2u) ? 2u : 1u) << 24 | k << 28;
        ++n;
    }
    if (n) {
        chk(hipMemcpyAsync(flags + kMaxDense, tab, sizeof tab, hipMemcpyHostToDevice, st));
        chk(hipStreamSynchronize(st));
        if (e != hipSuccess) return fail(PS_EDEVICE, "dense maps: %s", hipGetErrorString(e));
    }
    DevIndex& d = ix->dev;
    d.dense_tab = flags + kMaxDense;
    d.dense_maps = (const uint8_t*)(base + lay.dense);
    d.dense_stride = lay.dense_stride;
    ix->n_dense = n;
    bind_dense(ix);
    return PS_OK;
}

}  // namespace ps

extern "C" int ps_index_build_device_bytes(const ps_db_params* params, const char* residues, const uint64_t* prot_off,
                                           uint64_t n_proteins, uint64_t chunk_pairs_cap, uint64_t* index_bytes,
                                           uint64_t* scratch_bytes) {
    if (!index_bytes || !scratch_bytes) return fail(PS_EINVAL, "NULL argument");
    ps_index* ix = nullptr;
    int rc = index_prepare(params, residues, prot_off, n_proteins, &ix);
    if (rc != PS_OK) return rc;
    Census C;
    rc = census(ix, C);
    if (rc == PS_OK) rc = require_device();
    if (rc == PS_OK) {
        hipError_t e;
        const uint64_t chunk = chunk_pairs(C, chunk_pairs_cap, 2u * ix->merge_tol + 1u);
        const uint64_t tb = temp_bytes_for(C, chunk, nullptr, &e);
        if (e != hipSuccess) rc = fail(PS_EDEVICE, "sort workspace query: %s", hipGetErrorString(e));
        *index_bytes = index_layout(C.D, C.n_bins, C.quad_cap, C.n_bins * C.dir_stride, true, kMaxDense).total;
        *scratch_bytes = layout_scratch(nullptr, ix, C, chunk, tb).total;
    }
    delete ix;
    return rc;
}

extern "C" int ps_index_build_device(const ps_db_params* params, const char* residues, const uint64_t* prot_off,
                                     uint64_t n_proteins, uint64_t chunk_pairs_cap, const ps_device* index_block,
                                     const ps_device* scratch, ps_index** out) {
    if (!out) return fail(PS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!index_block || !scratch) return fail(PS_EINVAL, "NULL device block");
    ps_index* ix = nullptr;
    int rc = index_prepare(params, residues, prot_off, n_proteins, &ix);
    if (rc != PS_OK) return rc;
    hipStream_t st = (hipStream_t)index_block->stream;
    bool queued = false;                  // work on `st` may read host buffers of this function
    auto bail = [&](int code) {
        if (queued) (void)hipStreamSynchronize(st);
        delete ix;
        return code;
    };
    rc = require_device();
    if (rc != PS_OK) return bail(rc);
    Census C;
    rc = census(ix, C);
    if (rc != PS_OK) return bail(rc);
    hipError_t e = hipSuccess;
    const uint64_t chunk = chunk_pairs(C, chunk_pairs_cap, 2u * ix->merge_tol + 1u);
    const uint64_t tb = temp_bytes_for(C, chunk, st, &e);
    if (e != hipSuccess) return bail(fail(PS_EDEVICE, "sort workspace query: %s", hipGetErrorString(e)));
    const DevLayout lay = index_layout(C.D, C.n_bins, C.quad_cap, C.n_bins * C.dir_stride, true, kMaxDense);
    const Scratch need = layout_scratch(nullptr, ix, C, chunk, tb);
    if (!index_block->base || index_block->bytes < lay.total)
        return bail(fail(PS_ENOMEM, "index needs %llu device bytes, block has %llu", (unsigned long long)lay.total,
                         (unsigned long long)index_block->bytes));
    if (!scratch->base || scratch->bytes < need.total)
        return bail(fail(PS_ENOMEM, "index build needs %llu scratch bytes, block has %llu",
                         (unsigned long long)need.total, (unsigned long long)scratch->bytes));
    if (((uintptr_t)index_block->base & 255u) || ((uintptr_t)scratch->base & 255u))
        return bail(fail(PS_EINVAL, "device blocks must be 256-byte aligned"));
    char* base = (char*)index_block->base;
    Scratch S = layout_scratch((char*)scratch->base, ix, C, chunk, tb);
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    const ModTable mt = mod_table(ix);
    ModArgs M{};
    for (int i = 0; i < 26; ++i) M.res_mod[i] = mt.res_mod[i];
    M.nterm_mod = mt.nterm_mod;
    for (size_t m = 0; m < ix->mods.size(); ++m) M.delta[m] = ix->mods[m].delta;
    int64_t* mass = (int64_t*)(base + lay.mass);
    // the partition's entry table is written straight into the index block
    S.l_prot = (uint32_t*)(base + lay.prot);
    S.l_start = (uint32_t*)(base + lay.start);
    S.l_len = (uint8_t*)(base + lay.len);
    S.l_mask = (uint64_t*)(base + lay.mask);
    uint32_t* bin_q = (uint32_t*)(base + lay.bin);
    uint32_t* post = (uint32_t*)(base + lay.post);
    uint32_t* dir = (uint32_t*)(base + lay.dir);
    const uint64_t n_prot = ix->prot_off.size() - 1;

    // inputs
    queued = true;
    chk(hipMemcpyAsync(S.seq, ix->seq.data(), ix->seq.size(), hipMemcpyHostToDevice, st));
    chk(hipMemcpyAsync(S.prot_off, ix->prot_off.data(), (n_prot + 1) * 8, hipMemcpyHostToDevice, st));
    const uint64_t n_starts = C.st_prot.size();
    if (n_starts) {
        chk(hipMemcpyAsync(S.st_prot, C.st_prot.data(), n_starts * 4, hipMemcpyHostToDevice, st));
        chk(hipMemcpyAsync(S.st_pos, C.st_pos.data(), n_starts * 4, hipMemcpyHostToDevice, st));
        chk(hipMemcpyAsync(S.st_off, C.st_off.data(), (n_starts + 1) * 8, hipMemcpyHostToDevice, st));
    }
    chk(hipMemsetAsync(S.bad, 0, sizeof(int), st));
    // 2. entries
    if (e == hipSuccess && C.D_all > 0) {
        GenArgs g{S.seq, S.prot_off, S.st_prot, S.st_pos, S.st_off, n_starts, ix->missed, ix->min_len, ix->max_len,
                  ix->max_mods, M, C.min_mass, S.g_mass, S.g_prot, S.g_start, S.g_len, S.g_mask, S.key0, S.idx0};
        hipLaunchKernelGGL(k_gen_entries, dim3(grid_for(n_starts, 64)), dim3(64), 0, st, g);
        chk(hipGetLastError());
    }
    // 3. stable sort by mass; the partition takes every G-th rank
    const uint32_t* order = S.idx0;
    if (e == hipSuccess && C.D_all > 1) {
        hipcub::DoubleBuffer<uint64_t> keys(S.key0, S.key1);
        hipcub::DoubleBuffer<uint32_t> vals(S.idx0, S.idx1);
        size_t tbytes = S.temp_bytes;
        chk(hipcub::DeviceRadixSort::SortPairs(S.temp, tbytes, keys, vals, (int)C.D_all, 0,
                                               (int)bit_length((uint64_t)(C.max_mass - C.min_mass)), st));
        order = vals.Current();
    }
    const uint32_t width = 2u * ix->merge_tol + 1u;
    if (e == hipSuccess) {
        TakeArgs t{order, C.D, ix->n_shards, ix->shard, S.g_mass, S.g_prot, S.g_start, S.g_len, S.g_mask,
                   mass, S.l_prot, S.l_start, S.l_len, S.l_mask, S.pair_cnt,
                   width * (uint32_t)__builtin_popcount(ix->ion_types)};
        hipLaunchKernelGGL(k_take, dim3(grid_for(C.D + 1)), dim3(256), 0, st, t);
        chk(hipGetLastError());
    }
    // 4. ions: entry pair offsets, then chunks of (bin, posting) pairs
    IonArgs io{S.seq, S.prot_off, S.l_prot, S.l_start, S.l_len, S.l_mask, M, ion_series(ix->ion_types),
               (int32_t)ix->merge_tol, C.n_bins, 0, C.D, S.pair_off, nullptr, nullptr, S.bad};
    if (e == hipSuccess) {
        size_t tbytes = S.temp_bytes;
        chk(hipcub::DeviceScan::ExclusiveSum(S.temp, tbytes, S.pair_cnt, S.pair_off, (int)(C.D + 1), st));
    }
    std::vector<uint64_t> poff(C.D + 1);
    chk(hipMemcpyAsync(poff.data(), S.pair_off, (C.D + 1) * 8, hipMemcpyDeviceToHost, st));
    chk(hipStreamSynchronize(st));
    if (e != hipSuccess) return bail(fail(PS_EDEVICE, "index build: %s", hipGetErrorString(e)));
    const uint64_t n_post = poff[C.D];
    if (n_post > C.post_cap)
        return bail(fail(PS_EOVERFLOW, "postings exceed the computed bound (%llu > %llu)",
                         (unsigned long long)n_post, (unsigned long long)C.post_cap));
    // chunks of whole entries holding at most `chunk` pairs each
    std::vector<uint64_t> cuts{0};
    while (cuts.back() < C.D) {
        const uint64_t r0 = cuts.back();
        uint64_t r1 = (uint64_t)(std::upper_bound(poff.begin() + r0, poff.end(), poff[r0] + chunk) - poff.begin()) - 1;
        if (r1 <= r0) r1 = r0 + 1;                       // one entry never exceeds a chunk
        cuts.push_back(r1);
    }
    const size_t n_chunks = cuts.size() - 1;
    // generate and stably sort one chunk's pairs; returns the sorted buffers
    auto sorted_chunk = [&](size_t c, uint64_t& m) {
        const uint64_t r0 = cuts[c], r1 = cuts[c + 1];
        m = poff[r1] - poff[r0];
        io.r0 = r0; io.r1 = r1; io.key = S.pk0; io.val = S.pv0;
        hipLaunchKernelGGL(k_ions, dim3(grid_for(r1 - r0)), dim3(256), 0, st, io);
        chk(hipGetLastError());
        hipcub::DoubleBuffer<uint32_t> keys(S.pk0, S.pk1);
        hipcub::DoubleBuffer<uint32_t> vals(S.pv0, S.pv1);
        size_t tbytes = S.temp_bytes;
        if (m > 1) chk(hipcub::DeviceRadixSort::SortPairs(S.temp, tbytes, keys, vals, (int)m, 0,
                                                        (int)bit_length(C.n_bins), st));
        return std::make_pair(keys.Current(), vals.Current());
    };
    // pass 1: postings per bin, over every chunk (a single chunk stays sorted for pass 2)
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(C.n_bins + 1)), dim3(256), 0, st, S.bin_cnt, C.n_bins + 1);
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(C.n_bins)), dim3(256), 0, st, S.cursor, C.n_bins);
    uint64_t m_one = 0;
    std::pair<uint32_t*, uint32_t*> kv_one{S.pk0, S.pv0};
    for (size_t c = 0; c < n_chunks && e == hipSuccess; ++c) {
        uint64_t m = 0;
        auto kv = sorted_chunk(c, m);
        if (n_chunks == 1) { kv_one = kv; m_one = m; }
        hipLaunchKernelGGL(k_bin_runs, dim3(grid_for(C.n_bins)), dim3(256), 0, st, kv.first, m, C.n_bins, S.bin_cnt);
        chk(hipGetLastError());
    }
    // list offsets on the host: the plain CSR offsets (the index's host view) and
    // each list's first quad on the device, lists padded to whole quads
    std::vector<unsigned long long> cnt(C.n_bins);
    if (C.n_bins) chk(hipMemcpyAsync(cnt.data(), S.bin_cnt, C.n_bins * 8, hipMemcpyDeviceToHost, st));
    chk(hipStreamSynchronize(st));
    if (e != hipSuccess) return bail(fail(PS_EDEVICE, "index build: %s", hipGetErrorString(e)));
    std::vector<uint64_t> csr(C.n_bins + 1);
    std::vector<uint32_t> bq(C.n_bins + 1);
    uint64_t quads = 0;
    for (uint64_t b = 0; b < C.n_bins; ++b) {
        csr[b] = b ? csr[b - 1] + cnt[b - 1] : 0;
        if (cnt[b] >= (1ull << 32))
            return bail(fail(PS_EOVERFLOW, "fragment bin %llu holds 2^32 or more postings", (unsigned long long)b));
        bq[b] = (uint32_t)quads;
        quads += (cnt[b] + 3) >> 2;
        if (quads >= kMaxQuads)
            return bail(fail(PS_EOVERFLOW, "the postings need more than 2^32 16-byte quads"));
    }
    csr[C.n_bins] = C.n_bins ? csr[C.n_bins - 1] + cnt[C.n_bins - 1] : 0;
    bq[C.n_bins] = (uint32_t)quads;
    if (csr[C.n_bins] != n_post || quads > C.quad_cap)
        return bail(fail(PS_EDEVICE, "index build: inconsistent posting counts"));
    chk(hipMemcpyAsync(bin_q, bq.data(), (C.n_bins + 1) * 4, hipMemcpyHostToDevice, st));
    if (quads) {
        hipLaunchKernelGGL(k_fill_post, dim3(grid_for(quads * 4)), dim3(256), 0, st, post, kPostPad, quads * 4);
        chk(hipGetLastError());
    }
    // pass 2: scatter every chunk's runs behind the cursors
    for (size_t c = 0; c < n_chunks && e == hipSuccess; ++c) {
        uint64_t m = m_one;
        auto kv = n_chunks == 1 ? kv_one : sorted_chunk(c, m);
        if (m == 0) continue;
        ScatterArgs sa{kv.first, kv.second, m, S.run_start, S.run_end, bin_q, S.cursor, post};
        hipLaunchKernelGGL(k_runs, dim3(grid_for(m)), dim3(256), 0, st, sa);
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(m)), dim3(256), 0, st, sa);
        hipLaunchKernelGGL(k_advance, dim3(grid_for(m)), dim3(256), 0, st, sa);
        chk(hipGetLastError());
    }
    int bad = 0;
    chk(hipMemcpyAsync(&bad, S.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    chk(hipStreamSynchronize(st));
    if (e != hipSuccess) return bail(fail(PS_EDEVICE, "index build: %s", hipGetErrorString(e)));
    if (bad & 1) return bail(fail(PS_EINVAL, "a fragment ion has a negative mass (modification deltas too negative)"));
    if (bad & 2) return bail(fail(PS_EINVAL, "a fragment ion lies outside the bin range"));
    // 5. directory
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_dir, dim3(grid_for(C.n_bins * C.dir_stride)), dim3(256), 0, st, bin_q, S.bin_cnt,
                           post, C.n_bins, C.dir_stride, C.dir_shift, dir);
        chk(hipGetLastError());
    }
    // score tables; the host keeps only the bin offsets (the entry table stays
    // on the device, where ps_index_entry and ps_peptide read it back)
    std::vector<double> lf, ls;
    score_tables(lf, ls);
    chk(hipMemcpyAsync(base + lay.lf, lf.data(), lf.size() * 8, hipMemcpyHostToDevice, st));
    chk(hipMemcpyAsync(base + lay.ls, ls.data(), ls.size() * 8, hipMemcpyHostToDevice, st));
    ix->bin_off.swap(csr);
    chk(hipStreamSynchronize(st));
    if (e != hipSuccess) return bail(fail(PS_EDEVICE, "index build: %s", hipGetErrorString(e)));
    ix->n_bins = C.n_bins;
    ix->max_len_seen = C.max_len;
    ix->min_residue = lightest_residue(ix, mt);
    ix->dir_shift = C.dir_shift;
    ix->dir_nblk = C.dir_nblk;
    ix->dir_stride = C.dir_stride;
    ix->device_built = true;
    ix->n_entries = C.D;
    ix->dev_prot = S.l_prot;
    ix->dev_start = S.l_start;
    ix->dev_len = S.l_len;
    ix->dev_mask = S.l_mask;
    ix->dev_n_post = n_post;
    ix->dev_n_quads = quads;
    ix->dev_dir_entries = C.n_bins * C.dir_stride;
    bind_device_index(ix, base, lay);
    rc = build_dense_maps(ix, base, lay, st);
    if (rc != PS_OK) return bail(rc);
    if (ix->sched.tile < (1u << ix->dir_shift)) ix->sched.tile = 1u << ix->dir_shift;
    *out = ix;
    return PS_OK;
}

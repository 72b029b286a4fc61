// index.cpp -- host-side database construction and upload of the fragment-ion index.
//
// Superstep 1 of HiCOPS (arXiv 2102.02286; Supplementary Algorithm 1): generate
// every database entry (tryptic peptides and their modified forms, D = zeta*2^m
// in the paper's notation), sort them, generate b/y model spectra, and build a
// fragment-ion index.  The paper uses the CFIR-Index without printing its
// layout; this one is a CSR over 0.01-Da fragment bins whose postings hold the
// peptide id (= rank in the sorted entry order) and a b/y bit, sorted by id
// within each bin, so a precursor window is one contiguous sub-range per bin.
#include "state.h"
#include "batch.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <thread>

namespace ps {

static const int64_t kResidueUda[26] = {
    71037114, -1, 103009185, 115026943, 129042593, 147068414, 57021464, 137058912,   // A..H
    113084064, -1, 128094963, 113084064, 131040485, 114042927, -1, 97052764,         // I..P
    128058578, 156101111, 87032028, 101047679, -1, 99068414, 186079313, -1,          // Q..X
    163063329, -1,                                                                     // Y, Z
};

int64_t residue_uda(char c) {
    if (c < 'A' || c > 'Z') return -1;
    return kResidueUda[c - 'A'];
}

unsigned worker_threads() {
    unsigned t = std::thread::hardware_concurrency();
    if (t == 0) t = 4;
    return std::min(t, 32u);
}

template <typename F>
static void parallel_for(uint64_t n, unsigned threads, F&& f) {
    if (threads <= 1 || n < 2) { f(0, 0, n); return; }
    std::vector<std::thread> th;
    uint64_t chunk = (n + threads - 1) / threads;
    for (unsigned t = 0; t < threads; ++t) {
        uint64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([&f, t, a, b] { f(t, a, b); });
    }
    for (auto& x : th) x.join();
}

namespace {

struct PepRec {
    int64_t mass;
    uint32_t prot, start;
    uint32_t len, pad;
    uint64_t mask;
};

inline bool key_less(const PepRec& x, const PepRec& y) {
    if (x.mass != y.mass) return x.mass < y.mass;
    if (x.prot != y.prot) return x.prot < y.prot;
    if (x.start != y.start) return x.start < y.start;
    if (x.len != y.len) return x.len < y.len;
    return x.mask < y.mask;
}

// Sort in parallel: sorted chunks, then rounds of pairwise merges.
void parallel_sort(std::vector<PepRec>& v, unsigned threads) {
    uint64_t n = v.size();
    if (threads <= 1 || n < (1u << 16)) { std::sort(v.begin(), v.end(), key_less); return; }
    std::vector<uint64_t> bounds;
    for (unsigned t = 0; t <= threads; ++t) bounds.push_back(n * t / threads);
    parallel_for(threads, threads, [&](unsigned, uint64_t a, uint64_t b) {
        for (uint64_t t = a; t < b; ++t) std::sort(v.begin() + bounds[t], v.begin() + bounds[t + 1], key_less);
    });
    std::vector<PepRec> tmp(n);
    while (bounds.size() > 2) {
        std::vector<uint64_t> nb;
        uint64_t pairs = (bounds.size() - 1) / 2;
        std::vector<std::thread> th;
        for (uint64_t p = 0; p < pairs; ++p) {
            uint64_t a = bounds[2 * p], m = bounds[2 * p + 1], b = bounds[2 * p + 2];
            th.emplace_back([&, a, m, b] {
                std::merge(v.begin() + a, v.begin() + m, v.begin() + m, v.begin() + b, tmp.begin() + a, key_less);
            });
            nb.push_back(a);
        }
        for (auto& x : th) x.join();
        if ((bounds.size() - 1) % 2) {   // odd chunk out: copy it over
            uint64_t a = bounds[bounds.size() - 2], b = bounds.back();
            std::copy(v.begin() + a, v.begin() + b, tmp.begin() + a);
            nb.push_back(a);
        }
        nb.push_back(n);
        v.swap(tmp);
        bounds.swap(nb);
    }
}

}  // namespace

ModTable mod_table(const ps_index* ix) {
    ModTable t;
    for (int i = 0; i < 26; ++i) t.res_mod[i] = -1;
    t.nterm_mod = -1;
    for (size_t m = 0; m < ix->mods.size(); ++m) {
        if (ix->mods[m].nterm) t.nterm_mod = (int)m;
        else for (int i = 0; i < 26; ++i) if (ix->mods[m].res_mask >> i & 1u) t.res_mod[i] = (int)m;
    }
    return t;
}

// Residue masses of entry `id` with its modifications folded in; returns length.
static uint32_t entry_residues(const ps_index* ix, const ModTable& mt, uint64_t id, int64_t* r) {
    const char* s = ix->seq.data() + ix->prot_off[ix->prot[id]] + ix->start[id];
    uint32_t len = ix->len[id];
    uint64_t mask = ix->mask[id];
    uint32_t bit = 0;
    if (ix->start[id] == 0 && mt.nterm_mod >= 0) {
        r[0] = 0;   // filled below; the N-terminal site is bit 0
        if (mask & 1ull) r[0] += ix->mods[mt.nterm_mod].delta;
        bit = 1;
    } else {
        r[0] = 0;
    }
    for (uint32_t j = 0; j < len; ++j) {
        int64_t m = kResidueUda[s[j] - 'A'];
        int mm = mt.res_mod[s[j] - 'A'];
        if (mm >= 0) {
            if (mask >> bit & 1ull) m += ix->mods[mm].delta;
            ++bit;
        }
        if (j == 0) r[0] += m; else r[j] = m;
    }
    return len;
}

int index_build_host(ps_index* ix) {
    const unsigned T = worker_threads();
    const ModTable mt = mod_table(ix);
    const uint64_t n_prot = ix->prot_off.size() - 1;

    // 1. generate entries, per protein, in parallel
    std::vector<std::vector<PepRec>> parts(T);
    std::atomic<int> too_many{0};
    parallel_for(n_prot, T, [&](unsigned t, uint64_t pa, uint64_t pb) {
        auto& out = parts[t];
        int64_t site_delta[64];
        for (uint64_t p = pa; p < pb; ++p) {
            const char* s = ix->seq.data() + ix->prot_off[p];
            uint64_t n = ix->prot_off[p + 1] - ix->prot_off[p];
            for (uint64_t a = 0; a < n; ++a) {
                if (a != 0 && !is_cut(s, n, a - 1)) continue;
                uint32_t missed = 0;
                int64_t base = kWaterUda;
                for (uint64_t e = a + 1; e <= n; ++e) {
                    uint64_t len = e - a;
                    if (len > ix->max_len) break;
                    base += kResidueUda[s[e - 1] - 'A'];
                    bool end = (e == n) || is_cut(s, n, e - 1);
                    if (!end) continue;
                    if (len >= ix->min_len) {
                        // sites in mask-bit order
                        uint32_t ns = 0;
                        if (a == 0 && mt.nterm_mod >= 0) site_delta[ns++] = ix->mods[mt.nterm_mod].delta;
                        for (uint64_t j = a; j < e; ++j) {
                            int mm = mt.res_mod[s[j] - 'A'];
                            if (mm >= 0) site_delta[ns++] = ix->mods[mm].delta;
                        }
                        if (ns > 63) { too_many = 1; continue; }
                        // all subsets with <= max_mods sites: walk combinations by size
                        uint32_t kmax = std::min<uint32_t>(ix->max_mods, ns);
                        for (uint32_t k = 0; k <= kmax; ++k) {
                            uint32_t idx[64];
                            for (uint32_t i = 0; i < k; ++i) idx[i] = i;
                            while (true) {
                                PepRec r;
                                r.prot = (uint32_t)p; r.start = (uint32_t)a; r.len = (uint32_t)len; r.pad = 0;
                                r.mask = 0; r.mass = base;
                                for (uint32_t i = 0; i < k; ++i) { r.mask |= 1ull << idx[i]; r.mass += site_delta[idx[i]]; }
                                out.push_back(r);
                                // next combination
                                int i = (int)k - 1;
                                while (i >= 0 && idx[i] == ns - k + (uint32_t)i) --i;
                                if (i < 0) break;
                                ++idx[i];
                                for (uint32_t j = (uint32_t)i + 1; j < k; ++j) idx[j] = idx[j - 1] + 1;
                            }
                        }
                    }
                    if (e < n && ++missed > ix->missed) break;
                }
            }
        }
    });
    if (too_many) return fail(PS_EINVAL, "a peptide has more than 63 modifiable sites");
    uint64_t D = 0;
    for (auto& v : parts) D += v.size();
    if (D >= (1ull << 31)) return fail(PS_EOVERFLOW, "%llu database entries exceed the 2^31 id space",
                                       (unsigned long long)D);
    std::vector<PepRec> all;
    all.reserve(D);
    for (auto& v : parts) { all.insert(all.end(), v.begin(), v.end()); std::vector<PepRec>().swap(v); }

    // 2. sort by (mass, protein, start, length, mask): id = rank.  A partition
    //    keeps the ranks r with r % G == g (round-robin scatter of the sorted
    //    database); its entry r / G is entry r of the whole.  The longest
    //    peptide and the heaviest mass are taken over the whole database, so
    //    counter bounds and bin ranges match an unpartitioned index.
    parallel_sort(all, T);
    uint32_t max_len_seen = 0;
    int64_t max_mass = 0;
    for (uint64_t i = 0; i < D; ++i) {
        max_len_seen = std::max(max_len_seen, all[i].len);
        max_mass = std::max(max_mass, all[i].mass);
    }
    const uint64_t G = ix->n_shards, g = ix->shard;
    const uint64_t D_all = D;
    D = D_all > g ? (D_all - g + G - 1) / G : 0;
    ix->mass.resize(D); ix->prot.resize(D); ix->start.resize(D); ix->len.resize(D); ix->mask.resize(D);
    ix->n_entries = D;
    for (uint64_t i = 0; i < D; ++i) {
        const PepRec& r = all[i * G + g];
        ix->mass[i] = r.mass; ix->prot[i] = r.prot; ix->start[i] = r.start;
        ix->len[i] = (uint8_t)r.len; ix->mask[i] = r.mask;
    }
    std::vector<PepRec>().swap(all);
    ix->max_len_seen = max_len_seen;

    ix->min_residue = lightest_residue(ix, mt);

    // 3. b/y ion bins, two passes: count per (thread chunk, bin), then scatter in id order
    uint64_t nbins = (uint64_t)((max_mass + kBinWidth / 2) / kBinWidth) + 2;
    // a fragment bin is carried in 24 bits by the search kernels (167 kDa)
    if (nbins >= (1ull << 24)) return fail(PS_EOVERFLOW, "peptide masses need %llu fragment bins (limit 2^24)",
                                           (unsigned long long)nbins);
    ix->n_bins = nbins;
    std::vector<std::vector<uint32_t>> cnt(T);
    std::atomic<int> bad_mass{0};
    const IonSeries ions = ion_series(ix->ion_types);
    parallel_for(D, T, [&](unsigned t, uint64_t a, uint64_t b) {
        auto& c = cnt[t];
        c.assign(nbins, 0);
        int64_t r[64];
        for (uint64_t id = a; id < b; ++id) {
            uint32_t n = entry_residues(ix, mt, id, r);
            int64_t pre = 0, suf = 0;
            for (uint32_t i = 1; i < n; ++i) {
                pre += r[i - 1];
                suf += r[n - i];
                for (int t = 0; t < ions.n; ++t) {
                    const int64_t m = (ions.cterm[t] ? suf + kWaterUda : pre) + kProtonUda + ions.shift[t];
                    if (m < 0) { bad_mass = 1; continue; }
                    c[(uint64_t)((m + kBinWidth / 2) / kBinWidth)]++;
                }
            }
        }
    });
    if (bad_mass) return fail(PS_EINVAL, "a fragment ion has a negative mass (modification deltas too negative)");
    ix->bin_off.assign(nbins + 1, 0);
    uint64_t run = 0;
    std::vector<std::vector<uint64_t>> pos(T);
    for (unsigned t = 0; t < T; ++t) pos[t].assign(cnt[t].empty() ? 0 : nbins, 0);
    for (uint64_t bn = 0; bn < nbins; ++bn) {
        ix->bin_off[bn] = run;
        for (unsigned t = 0; t < T; ++t) {
            if (cnt[t].empty()) continue;
            pos[t][bn] = run;
            run += cnt[t][bn];
        }
    }
    ix->bin_off[nbins] = run;
    for (auto& c : cnt) std::vector<uint32_t>().swap(c);
    ix->post.resize(run);
    parallel_for(D, T, [&](unsigned t, uint64_t a, uint64_t b) {
        auto& p = pos[t];
        int64_t r[64];
        for (uint64_t id = a; id < b; ++id) {
            uint32_t n = entry_residues(ix, mt, id, r);
            for (int t = 0; t < ions.n; ++t) {      // N-terminal series (bit 0) first, then C-terminal
                int64_t acc = 0;
                for (uint32_t i = 1; i < n; ++i) {
                    acc += ions.cterm[t] ? r[n - i] : r[i - 1];
                    const int64_t m = (ions.cterm[t] ? acc + kWaterUda : acc) + kProtonUda + ions.shift[t];
                    uint64_t bn = (uint64_t)((m + kBinWidth / 2) / kBinWidth);
                    ix->post[p[bn]++] = (uint32_t)(id << 1 | ions.cterm[t]);
                }
            }
        }
    });
    // Postings of one id in one bin must be ordered N-terminal before C-terminal; ions
    // of one id are emitted that way, so each bin is non-decreasing in (id << 1 | type).

    // 4. with a merge width T, the list of bin b becomes the id-ordered merge of
    // the lists of bins b-T..b+T: a peak then probes one list and still meets
    // every ion within T bins once
    if (ix->merge_tol > 0) {
        const int64_t mt = ix->merge_tol;
        std::vector<uint64_t> off2(nbins + 1, 0);
        for (uint64_t bn = 0; bn < nbins; ++bn) {
            const uint64_t a = (uint64_t)std::max<int64_t>(0, (int64_t)bn - mt);
            const uint64_t b = std::min<uint64_t>(nbins, bn + mt + 1);
            off2[bn + 1] = off2[bn] + (ix->bin_off[b] - ix->bin_off[a]);
        }
        std::vector<uint32_t> post2(off2[nbins]);
        parallel_for(nbins, T, [&](unsigned, uint64_t ba, uint64_t bb) {
            std::vector<uint32_t> tmp;
            for (uint64_t bn = ba; bn < bb; ++bn) {
                const uint64_t a = (uint64_t)std::max<int64_t>(0, (int64_t)bn - mt);
                const uint64_t b = std::min<uint64_t>(nbins, bn + mt + 1);
                uint32_t* dst = post2.data() + off2[bn];
                // each source list is sorted; merge them pairwise in order
                uint64_t filled = 0;
                for (uint64_t src = a; src < b; ++src) {
                    const uint32_t* p0 = ix->post.data() + ix->bin_off[src];
                    const uint64_t n0 = ix->bin_off[src + 1] - ix->bin_off[src];
                    tmp.resize(filled + n0);
                    std::merge(dst, dst + filled, p0, p0 + n0, tmp.begin());
                    std::copy(tmp.begin(), tmp.end(), dst);
                    filled += n0;
                }
            }
        });
        ix->bin_off.swap(off2);
        ix->post.swap(post2);
    }

    // 5. tile directory: for every bin and every block of 2^dir_shift ids, the
    // position in the bin's list of its first posting at or after the block
    // start.  A scan tile is a whole number of blocks, so every posting run's
    // tile boundaries are direct lookups.  The grain is 4096 ids unless the
    // directory would pass kDirBudget bytes.
    for (uint64_t bn = 0; bn < nbins; ++bn)
        if (ix->bin_off[bn + 1] - ix->bin_off[bn] >= (1ull << 32))
            return fail(PS_EOVERFLOW, "fragment bin %llu holds 2^32 or more postings", (unsigned long long)bn);
    if (padded_quads(ix) >= kMaxQuads)
        return fail(PS_EOVERFLOW, "the postings need %llu 16-byte quads; at most 2^32 are addressable",
                    (unsigned long long)padded_quads(ix));
    ix->dir_shift = directory_shift(nbins, D);
    // Rows are padded to a multiple of four entries (16 bytes), so a row can be
    // read four tile boundaries at a time; padding repeats the bin's end.
    ix->dir_nblk = (D >> ix->dir_shift) + 1;
    ix->dir_stride = (ix->dir_nblk + 1 + 3) & ~3ull;
    const uint64_t stride = ix->dir_stride;
    ix->dir.assign(nbins * stride, 0u);
    parallel_for(nbins, T, [&](unsigned, uint64_t ba, uint64_t bb) {
        for (uint64_t bn = ba; bn < bb; ++bn) {
            uint32_t* d = ix->dir.data() + bn * stride;
            const uint64_t b0 = ix->bin_off[bn];
            uint64_t i = b0;
            const uint64_t e = ix->bin_off[bn + 1];
            for (uint64_t k = 0; k < stride; ++k) {
                const uint64_t first_id = k << ix->dir_shift;
                while (i < e && (uint64_t)(ix->post[i] >> 1) < first_id) ++i;
                d[k] = (uint32_t)(i - b0);
            }
        }
    });
    return PS_OK;
}

// lightest residue including modification deltas (bounds how many ions of one
// peptide can share a tolerance window)
int64_t lightest_residue(const ps_index* ix, const ModTable& mt) {
    int64_t nterm_neg = mt.nterm_mod >= 0 ? std::min<int64_t>(0, ix->mods[mt.nterm_mod].delta) : 0;
    int64_t minres = INT64_MAX;
    for (int c = 0; c < 26; ++c) {
        if (kResidueUda[c] < 0) continue;
        int64_t m = kResidueUda[c] + nterm_neg;
        if (mt.res_mod[c] >= 0) m += std::min<int64_t>(0, ix->mods[mt.res_mod[c]].delta);
        minres = std::min(minres, m);
    }
    return minres;
}

uint64_t padded_quads(const ps_index* ix) {
    if (ix->device_built) return ix->dev_n_quads;
    uint64_t q = 0;
    for (uint64_t b = 0; b + 1 < ix->bin_off.size(); ++b) q += (ix->bin_off[b + 1] - ix->bin_off[b] + 3) >> 2;
    return q;
}

uint32_t directory_shift(uint64_t nbins, uint64_t D) {
    constexpr uint64_t kDirBudget = 32ull << 30;
    uint32_t sh = 12;
    while (sh < 16 && nbins * ((D >> sh) + 6) * 4 > kDirBudget) ++sh;
    return sh;
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

DevLayout index_layout(uint64_t n_pep, uint64_t n_bins, uint64_t n_quads, uint64_t n_dir, bool entries,
                       uint32_t dense_cap) {
    DevLayout L;
    uint64_t o = 0;
    L.mass = o; o = align256(o + n_pep * sizeof(int64_t));
    L.bin = o; o = align256(o + (n_bins + 1) * sizeof(uint32_t));
    L.post = o; o = align256(o + n_quads * 16 + 16);
    L.lf = o; o = align256(o + kLfSize * sizeof(double));
    L.ls = o; o = align256(o + kLsSize * sizeof(double));
    L.dir = o; o = align256(o + n_dir * sizeof(uint32_t));
    const uint64_t ne = entries ? (n_pep > 0 ? n_pep : 1) : 0;
    L.prot = o; o = align256(o + ne * sizeof(uint32_t));
    L.start = o; o = align256(o + ne * sizeof(uint32_t));
    L.mask = o; o = align256(o + ne * sizeof(uint64_t));
    L.len = o; o = align256(o + ne);
    L.dense_cap = n_pep ? dense_cap : 0u;
    L.dense_stride = align256(dense_map_bytes(n_pep));
    L.dense = o; o = align256(o + (uint64_t)L.dense_cap * L.dense_stride);
    L.dense_flags = o; o = align256(o + 2 * kMaxDense * sizeof(uint32_t));
    L.total = o;
    return L;
}

std::vector<uint32_t> dense_candidates(const ps_index* ix) {
    std::vector<std::pair<uint64_t, uint32_t>> c;
    const uint64_t D = ix->n_entries;
    for (uint64_t b = 0; D && b + 1 < ix->bin_off.size(); ++b) {
        const uint64_t len = ix->bin_off[b + 1] - ix->bin_off[b];
        if (len * 4 >= D) c.push_back({len, (uint32_t)b});
    }
    std::sort(c.begin(), c.end(), [](const auto& a, const auto& b) { return a.first > b.first || (a.first == b.first && a.second < b.second); });
    std::vector<uint32_t> out;
    for (size_t i = 0; i < c.size() && i < kMaxDense; ++i) out.push_back(c[i].second);
    return out;
}

void bind_dense(ps_index* ix) {
    DevIndex& d = ix->dev;
    d.n_dense = ix->dense_on ? ix->n_dense : 0u;
}

static DevLayout index_device_layout(const ps_index* ix) {
    return index_layout(ix->n_entries, ix->n_bins, padded_quads(ix), dir_entries(ix), false,
                        (uint32_t)dense_candidates(ix).size());
}

void bind_device_index(ps_index* ix, char* base, const DevLayout& lay) {
    DevIndex& d = ix->dev;
    d.mass = (const int64_t*)(base + lay.mass);
    d.bin_q = (const uint32_t*)(base + lay.bin);
    d.post = (const uint32_t*)(base + lay.post);
    d.lf = (const double*)(base + lay.lf);
    d.ls = (const double*)(base + lay.ls);
    d.dir = (const uint32_t*)(base + lay.dir);
    d.dir_shift = ix->dir_shift;
    d.dir_nblk = (uint32_t)ix->dir_nblk;
    d.dir_stride = (uint32_t)ix->dir_stride;
    d.merge_tol = ix->merge_tol;
    d.n_pep = ix->n_entries;
    d.n_bins = ix->n_bins;
    d.n_post = n_postings(ix);
    d.max_len = ix->max_len_seen;
    d.ion_mult = ion_mult(ix->ion_types);
    d.ion_series = (uint32_t)__builtin_popcount(ix->ion_types);
    d.min_residue = ix->min_residue;
    ix->on_device = true;
}

void score_tables(std::vector<double>& lf, std::vector<double>& ls) {
    // hyperscore terms: lf[n] = sum_{k=2..n} log10 k accumulated left to right;
    // ls[s] = log10 s (ls[0] is never used: scored candidates have s >= 1)
    lf.assign(kLfSize, 0.0);
    double acc = 0.0;
    for (uint32_t k = 2; k < kLfSize; ++k) { acc += std::log10((double)k); lf[k] = acc; }
    ls.assign(kLsSize, 0.0);
    ls[0] = -INFINITY;
    for (uint32_t s = 1; s < kLsSize; ++s) ls[s] = std::log10((double)s);
}

}  // namespace ps

using namespace ps;

namespace ps {

// Validate the database parameters and make an index object holding them and the
// proteins, with nothing built yet.
int index_prepare(const ps_db_params* params, const char* residues, const uint64_t* prot_off,
                  uint64_t n_proteins, ps_index** out) {
    if (!out) return fail(PS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params || !residues || !prot_off) return fail(PS_EINVAL, "NULL argument");
    if (params->min_len < 2 || params->max_len < params->min_len || params->max_len > 62)
        return fail(PS_EINVAL, "peptide lengths must satisfy 2 <= min_len <= max_len <= 62");
    if (params->n_mods > 16) return fail(PS_EINVAL, "at most 16 modifications");
    if (params->n_mods && !params->mods) return fail(PS_EINVAL, "mods is NULL");
    if (prot_off[0] != 0) return fail(PS_EINVAL, "prot_off[0] must be 0");
    for (uint64_t i = 0; i < n_proteins; ++i)
        if (prot_off[i + 1] < prot_off[i]) return fail(PS_EINVAL, "prot_off must be non-decreasing");
    uint64_t total = prot_off[n_proteins];
    for (uint64_t i = 0; i < total; ++i)
        if (residue_uda(residues[i]) < 0)
            return fail(PS_EINVAL, "residue %llu ('%c') is not one of the 20 standard amino acids",
                        (unsigned long long)i, residues[i]);
    if (params->merge_tol_bins > PS_MAX_FRAG_TOL_BINS)
        return fail(PS_EINVAL, "merge_tol_bins must be 0..%d", PS_MAX_FRAG_TOL_BINS);
    const uint32_t n_shards = params->n_shards ? params->n_shards : 1u;
    if (n_shards > PS_MAX_SHARDS || params->shard >= n_shards)
        return fail(PS_EINVAL, "need shard < n_shards <= %d (got shard %u of %u)", PS_MAX_SHARDS,
                    params->shard, n_shards);
    if (params->ion_types > 63) return fail(PS_EINVAL, "ion_types must be a set of PS_ION_* bits");
    if (params->reserved != 0) return fail(PS_EINVAL, "reserved must be 0");
    ps_index* ix = new (std::nothrow) ps_index();
    if (!ix) return fail(PS_ENOMEM, "out of host memory");
    ix->ion_types = params->ion_types ? params->ion_types : (PS_ION_B | PS_ION_Y);
    ix->n_shards = n_shards;
    ix->shard = params->shard;
    ix->merge_tol = params->merge_tol_bins;
    ix->missed = params->missed_cleavages;
    ix->min_len = params->min_len;
    ix->max_len = params->max_len;
    ix->max_mods = params->max_mods;
    uint32_t letters_used = 0;
    int nterm_count = 0;
    for (uint32_t m = 0; m < params->n_mods; ++m) {
        const ps_mod& pm = params->mods[m];
        ps_index::Mod md;
        md.nterm = pm.nterm != 0;
        md.delta = pm.delta_udalton;
        md.res_mask = 0;
        if (md.nterm) {
            ++nterm_count;
        } else {
            if (!pm.residues || !pm.residues[0]) { delete ix; return fail(PS_EINVAL, "mod %u has no residues", m); }
            for (const char* c = pm.residues; *c; ++c) {
                if (residue_uda(*c) < 0) { delete ix; return fail(PS_EINVAL, "mod %u: bad residue '%c'", m, *c); }
                md.res_mask |= 1u << (*c - 'A');
            }
            if (md.res_mask & letters_used) { delete ix; return fail(PS_EINVAL, "a residue appears in two mods"); }
            letters_used |= md.res_mask;
            md.residues = pm.residues;
        }
        ix->mods.push_back(md);
    }
    if (nterm_count > 1) { delete ix; return fail(PS_EINVAL, "at most one N-terminal mod"); }
    // every residue, modified or not, must stay heavier than a proton plus the widest
    // fragment tolerance, so every b/y ion and its tolerance window lie inside the
    // bin range of the database's masses
    // (a and x ions lose or gain CO at the ends, so they need residues heavier than CO)
    const int64_t floor_uda = ((ix->ion_types & (PS_ION_A | PS_ION_X)) ? kCOUda : kProtonUda) +
                              kBinWidth * (PS_MAX_FRAG_TOL_BINS + 1);
    if (lightest_residue(ix, mod_table(ix)) <= floor_uda) {
        delete ix;
        return fail(PS_EINVAL, "a modification makes a residue lighter than %.3f Da", floor_uda * 1e-6);
    }
    try {
        ix->seq.assign(residues, residues + total);
        ix->prot_off.assign(prot_off, prot_off + n_proteins + 1);
    } catch (...) { delete ix; return fail(PS_ENOMEM, "out of host memory"); }
    ix->sched = default_schedule();
    *out = ix;
    return PS_OK;
}

}  // namespace ps

extern "C" int ps_index_create(const ps_db_params* params, const char* residues, const uint64_t* prot_off,
                               uint64_t n_proteins, ps_index** out) {
    ps_index* ix = nullptr;
    int rc = index_prepare(params, residues, prot_off, n_proteins, &ix);
    if (rc != PS_OK) { if (out) *out = nullptr; return rc; }
    try { rc = index_build_host(ix); } catch (...) { rc = fail(PS_ENOMEM, "out of host memory building the index"); }
    if (rc != PS_OK) { delete ix; *out = nullptr; return rc; }
    if (ix->sched.tile < (1u << ix->dir_shift)) ix->sched.tile = 1u << ix->dir_shift;
    *out = ix;
    return PS_OK;
}

extern "C" int ps_index_device_bytes(const ps_index* ix, uint64_t* bytes) {
    if (!ix || !bytes) return fail(PS_EINVAL, "NULL argument");
    *bytes = index_device_layout(ix).total;
    return PS_OK;
}

// Quad index of every bin's padded list, and the quad count last.
static std::vector<uint32_t> bin_quads(const ps_index* ix) {
    std::vector<uint32_t> q(ix->n_bins + 1);
    uint64_t run = 0;
    for (uint64_t b = 0; b < ix->n_bins; ++b) {
        q[b] = (uint32_t)run;
        run += (ix->bin_off[b + 1] - ix->bin_off[b] + 3) >> 2;
    }
    q[ix->n_bins] = (uint32_t)run;
    return q;
}

// Host postings into device memory with every bin's list padded to whole quads
// (filler kPostPad), through two pinned staging buffers so that filling one
// overlaps the copy of the other.
static hipError_t upload_padded_postings(const ps_index* ix, uint32_t* dst, hipStream_t st) {
    constexpr uint64_t kStage = 16ull << 20;             // entries per staging buffer (64 MB)
    uint32_t* buf[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    for (int i = 0; i < 2; ++i) {
        chk(hipHostMalloc((void**)&buf[i], kStage * 4, hipHostMallocDefault));
        chk(hipEventCreateWithFlags(&done[i], hipEventDisableTiming));
    }
    int cur = 0;
    uint64_t fill = 0, written = 0;
    bool pending[2] = {false, false};
    auto flush = [&]() {
        if (e != hipSuccess || fill == 0) return;
        chk(hipMemcpyAsync(dst + written, buf[cur], fill * 4, hipMemcpyHostToDevice, st));
        chk(hipEventRecord(done[cur], st));
        pending[cur] = true;
        written += fill;
        fill = 0;
        cur ^= 1;
        if (pending[cur]) { chk(hipEventSynchronize(done[cur])); pending[cur] = false; }
    };
    auto append = [&](const uint32_t* src, uint64_t n, uint32_t value) {
        while (n && e == hipSuccess) {
            const uint64_t m = std::min(n, kStage - fill);
            if (src) { memcpy(buf[cur] + fill, src, m * 4); src += m; }
            else std::fill(buf[cur] + fill, buf[cur] + fill + m, value);
            fill += m;
            n -= m;
            if (fill == kStage) flush();
        }
    };
    for (uint64_t b = 0; b < ix->n_bins && e == hipSuccess; ++b) {
        const uint64_t len = ix->bin_off[b + 1] - ix->bin_off[b];
        append(ix->post.data() + ix->bin_off[b], len, 0);
        append(nullptr, ((len + 3) & ~3ull) - len, kPostPad);
    }
    flush();
    for (int i = 0; i < 2; ++i) {
        if (pending[i]) chk(hipEventSynchronize(done[i]));
        if (done[i]) (void)hipEventDestroy(done[i]);
        if (buf[i]) (void)hipHostFree(buf[i]);
    }
    return e;
}

extern "C" int ps_index_upload(ps_index* ix, const ps_device* dev) {
    if (!ix || !dev) return fail(PS_EINVAL, "NULL argument");
    if (ix->device_built) return fail(PS_EINVAL, "this index was built on the device and is already there");
    int rc = require_device();
    if (rc != PS_OK) return rc;
    if (padded_quads(ix) >= kMaxQuads)
        return fail(PS_EOVERFLOW, "index needs %llu posting quads; at most 2^32 are addressable",
                    (unsigned long long)padded_quads(ix));
    const DevLayout lay = index_device_layout(ix);
    const uint64_t need = lay.total;
    if (!dev->base || dev->bytes < need)
        return fail(PS_ENOMEM, "index needs %llu device bytes, block has %llu", (unsigned long long)need,
                    (unsigned long long)dev->bytes);
    if (((uintptr_t)dev->base & 255u) != 0) return fail(PS_EINVAL, "device block must be 256-byte aligned");
    std::vector<double> lf, ls;
    score_tables(lf, ls);
    const std::vector<uint32_t> bq = bin_quads(ix);
    char* base = (char*)dev->base;
    hipStream_t st = (hipStream_t)dev->stream;
    hipError_t e = hipSuccess;
    auto cp = [&](uint64_t off, const void* src, size_t n) {
        if (e == hipSuccess && n) e = hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, st);
    };
    cp(lay.mass, ix->mass.data(), ix->mass.size() * sizeof(int64_t));
    cp(lay.bin, bq.data(), bq.size() * sizeof(uint32_t));
    cp(lay.lf, lf.data(), lf.size() * sizeof(double));
    cp(lay.ls, ls.data(), ls.size() * sizeof(double));
    cp(lay.dir, ix->dir.data(), ix->dir.size() * sizeof(uint32_t));
    if (e == hipSuccess) e = upload_padded_postings(ix, (uint32_t*)(base + lay.post), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(st);                  // queued copies read lf, ls and bq
        return fail(PS_EDEVICE, "index upload: %s", hipGetErrorString(e));
    }
    bind_device_index(ix, base, lay);
    rc = build_dense_maps(ix, base, lay, st);
    if (rc != PS_OK) { ix->on_device = false; return rc; }
    return PS_OK;
}

extern "C" int ps_build_index(const ps_device* dev, const ps_db_params* params, const char* residues,
                              const uint64_t* prot_off, uint64_t n_proteins, ps_index** out) {
    int rc = ps_index_create(params, residues, prot_off, n_proteins, out);
    if (rc != PS_OK) return rc;
    rc = ps_index_upload(*out, dev);
    if (rc != PS_OK) { ps_index_free(*out); *out = nullptr; }
    return rc;
}

extern "C" int ps_index_shape(const ps_index* ix, uint64_t* n_pep, uint64_t* n_post, uint64_t* n_bins) {
    if (!ix) return fail(PS_EINVAL, "NULL index");
    if (n_pep) *n_pep = ix->n_entries;
    if (n_post) *n_post = n_postings(ix);
    if (n_bins) *n_bins = ix->n_bins;
    return PS_OK;
}

// Entries [first, first + count) into host arrays (any may be NULL): from the
// host table, or read back from the device for an index built there.
static int read_entries(const ps_index* ix, uint64_t first, uint64_t count, int64_t* mass, uint32_t* protein,
                        uint32_t* start, uint8_t* length, uint64_t* site_mask) {
    if (!ix->device_built) {
        if (mass) memcpy(mass, ix->mass.data() + first, count * sizeof(int64_t));
        if (protein) memcpy(protein, ix->prot.data() + first, count * sizeof(uint32_t));
        if (start) memcpy(start, ix->start.data() + first, count * sizeof(uint32_t));
        if (length) memcpy(length, ix->len.data() + first, count);
        if (site_mask) memcpy(site_mask, ix->mask.data() + first, count * sizeof(uint64_t));
        return PS_OK;
    }
    if (count == 0) return PS_OK;
    hipError_t e = hipSuccess;
    auto get = [&](void* dst, const void* src, size_t elem) {
        if (dst && e == hipSuccess)
            e = hipMemcpy(dst, (const char*)src + first * elem, count * elem, hipMemcpyDeviceToHost);
    };
    get(mass, ix->dev.mass, sizeof(int64_t));
    get(protein, ix->dev_prot, sizeof(uint32_t));
    get(start, ix->dev_start, sizeof(uint32_t));
    get(length, ix->dev_len, 1);
    get(site_mask, ix->dev_mask, sizeof(uint64_t));
    return e == hipSuccess ? PS_OK : fail(PS_EDEVICE, "entries to host: %s", hipGetErrorString(e));
}

extern "C" int ps_index_entry(const ps_index* ix, uint64_t id, int64_t* mass, uint32_t* protein,
                              uint32_t* start, uint32_t* length, uint64_t* site_mask) {
    if (!ix) return fail(PS_EINVAL, "NULL index");
    if (id >= ix->n_entries) return fail(PS_EINVAL, "id %llu out of range", (unsigned long long)id);
    uint8_t len8 = 0;
    const int rc = read_entries(ix, id, 1, mass, protein, start, length ? &len8 : nullptr, site_mask);
    if (rc == PS_OK && length) *length = len8;
    return rc;
}

extern "C" int ps_index_entries(const ps_index* ix, uint64_t first, uint64_t count, int64_t* mass, uint32_t* protein,
                                uint32_t* start, uint8_t* length, uint64_t* site_mask) {
    if (!ix) return fail(PS_EINVAL, "NULL index");
    const uint64_t D = ix->n_entries;
    if (first > D || count > D - first)
        return fail(PS_EINVAL, "entries [%llu, %llu) out of range (%llu)", (unsigned long long)first,
                    (unsigned long long)(first + count), (unsigned long long)D);
    return read_entries(ix, first, count, mass, protein, start, length, site_mask);
}

extern "C" int ps_peptide(const ps_index* ix, uint32_t id, char* buf, size_t cap) {
    if (!ix || !buf || cap == 0) return fail(PS_EINVAL, "NULL argument");
    if (id >= ix->n_entries) return fail(PS_EINVAL, "id %u out of range", id);
    uint32_t prot = 0, start = 0;
    uint8_t len = 0;
    uint64_t mask = 0;
    const int rc = read_entries(ix, id, 1, nullptr, &prot, &start, &len, &mask);
    if (rc != PS_OK) return rc;
    ModTable mt = mod_table(ix);
    std::string s;
    const char* seq = ix->seq.data() + ix->prot_off[prot] + start;
    uint32_t bit = 0;
    char tmp[48];
    if (start == 0 && mt.nterm_mod >= 0) {
        if (mask & 1ull) {
            snprintf(tmp, sizeof tmp, "n[%+.6f]", ix->mods[mt.nterm_mod].delta * 1e-6);
            s += tmp;
        }
        bit = 1;
    }
    for (uint32_t j = 0; j < len; ++j) {
        s += seq[j];
        int mm = mt.res_mod[seq[j] - 'A'];
        if (mm >= 0) {
            if (mask >> bit & 1ull) {
                snprintf(tmp, sizeof tmp, "[%+.6f]", ix->mods[mm].delta * 1e-6);
                s += tmp;
            }
            ++bit;
        }
    }
    size_t n = std::min(cap - 1, s.size());
    memcpy(buf, s.data(), n);
    buf[n] = 0;
    return n < s.size() ? fail(PS_ENOMEM, "buffer too small for peptide string") : PS_OK;
}

extern "C" int ps_index_host_arrays(const ps_index* ix, uint64_t* bin_off, uint32_t* postings) {
    if (!ix) return fail(PS_EINVAL, "NULL index");
    if (bin_off) memcpy(bin_off, ix->bin_off.data(), ix->bin_off.size() * sizeof(uint64_t));
    if (postings && ix->device_built) {
        // the device lists are padded to whole quads: copy them, then close the gaps
        std::vector<uint32_t> padded;
        try { padded.resize(ix->dev_n_quads * 4); } catch (...) { return fail(PS_ENOMEM, "out of host memory"); }
        hipError_t e = hipMemcpy(padded.data(), ix->dev.post, padded.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail(PS_EDEVICE, "postings to host: %s", hipGetErrorString(e));
        uint64_t q = 0;
        for (uint64_t b = 0; b < ix->n_bins; ++b) {
            const uint64_t len = ix->bin_off[b + 1] - ix->bin_off[b];
            memcpy(postings + ix->bin_off[b], padded.data() + 4 * q, len * sizeof(uint32_t));
            q += (len + 3) >> 2;
        }
    } else if (postings) {
        memcpy(postings, ix->post.data(), ix->post.size() * sizeof(uint32_t));
    }
    return PS_OK;
}

extern "C" int ps_index_dense(const ps_index* ix, uint32_t* n_dense, uint32_t* bins, int* enabled) {
    if (!ix) return fail(PS_EINVAL, "NULL index");
    if (n_dense) *n_dense = ix->n_dense;
    if (bins) for (uint32_t k = 0; k < ix->n_dense; ++k) bins[k] = ix->dense_bin[k];
    if (enabled) *enabled = ix->dense_on ? 1 : 0;
    return PS_OK;
}

extern "C" int ps_index_set_dense(ps_index* ix, int enabled) {
    if (!ix) return fail(PS_EINVAL, "NULL index");
    ix->dense_on = enabled != 0;
    bind_dense(ix);
    return PS_OK;
}

extern "C" int ps_index_directory(const ps_index* ix, uint32_t* grain_shift, uint64_t* bytes, uint32_t* dir) {
    if (!ix) return fail(PS_EINVAL, "NULL index");
    if (grain_shift) *grain_shift = ix->dir_shift;
    if (bytes) *bytes = dir_entries(ix) * sizeof(uint32_t);
    if (dir && ix->device_built) {
        hipError_t e = hipMemcpy(dir, ix->dev.dir, ix->dev_dir_entries * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail(PS_EDEVICE, "directory to host: %s", hipGetErrorString(e));
    } else if (dir) {
        memcpy(dir, ix->dir.data(), ix->dir.size() * sizeof(uint32_t));
    }
    return PS_OK;
}

extern "C" void ps_index_free(ps_index* ix) { delete ix; }

// kernels.hip -- the search path on gfx950.
//
//   k_prep     spectrum pre-processing (top-B peaks, integer intensities, m/z to
//              uDa, fragment-charge expansion to bin entries) and the precursor
//              window (filter_1 of Supplementary Algorithm 3)
//   k_scan     per work item (spectrum, id range): fragment-bin lookups to
//              posting runs (filter_2), a load-balanced gather of each tile's
//              postings into LDS shared-peak counters, then per tile the
//              candidate filter (shared peaks >= k), hyperscore, wavefront
//              top-k and the LDS score histogram (Supplementary Algorithm 3's
//              score/heap)
//
// The statistics that follow the scan (merge of partial top-k lists, expect
// values, partition assembly and sampling) are in stats.hip.
//
// Integer work is exact: counters are packed integer fields, the histogram is
// integer, and hyperscores come from host-built fp64 tables, so results do not
// depend on atomic order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "internal.h"

namespace ps {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// llround for x >= 0: nearest integer, halves away from zero.
__device__ __forceinline__ int64_t round_half_up_pos(double x) {
    double t = trunc(x);
    return (int64_t)t + ((x - t) >= 0.5 ? 1 : 0);
}

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* a, uint32_t lo, uint32_t hi, uint32_t v) {
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <typename T, uint32_t NT = kBlock>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
    // scratch: NT/64 slots
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(NT / 64); ++i) r += scratch[i];
        scratch[0] = r;
    }
    __syncthreads();
    r = scratch[0];
    __syncthreads();
    return r;
}

// Packed shared-peak counters.  Narrow: [n_b + n_y : 9 | n_y : 8 | S : 15] in
// 32 bits, so that a candidate has at least k shared peaks exactly when its
// counter is at least k << 23 (one unsigned compare in the filter); wide:
// [n_b:16 | n_y:16 | S:32] in 64 bits.  The prep kernel proves per spectrum
// that no field can overflow before choosing the narrow form.  key(c) is
// monotone in n_b + n_y and key_min(k) its threshold for k shared peaks.
template <typename C> struct Cnt;
template <> struct Cnt<uint32_t> {
    __device__ static uint32_t inc(uint32_t is_y, uint32_t q) { return (1u << 23) + (is_y << 15) + q; }
    __device__ static uint32_t ny(uint32_t c) { return (c >> 15) & 0xFFu; }
    __device__ static uint32_t nb(uint32_t c) { return (c >> 23) - ny(c); }
    __device__ static uint32_t s(uint32_t c) { return c & 0x7FFFu; }
    __device__ static uint32_t key(uint32_t c) { return c; }
    // n_b + n_y <= 510: a threshold of 512 or more is never reached
    __device__ static uint32_t key_min(uint32_t k) { return k < 512u ? k << 23 : 0xFFFFFFFFu; }
};
template <> struct Cnt<unsigned long long> {
    __device__ static unsigned long long inc(uint32_t is_y, uint32_t q) {
        return (is_y ? (1ull << 32) : (1ull << 48)) + (unsigned long long)q;
    }
    __device__ static uint32_t nb(unsigned long long c) { return (uint32_t)(c >> 48); }
    __device__ static uint32_t ny(unsigned long long c) { return (uint32_t)(c >> 32) & 0xFFFFu; }
    __device__ static uint32_t s(unsigned long long c) { return (uint32_t)c; }
    __device__ static uint32_t key(unsigned long long c) { return nb(c) + ny(c); }
    __device__ static uint32_t key_min(uint32_t k) { return k; }
};

// Top-k of one wavefront, distributed over its lanes: lane j < k holds the
// j-th best candidate by (hyperscore desc, id asc).  An insertion is a ballot
// for the first lane the newcomer beats and a one-lane shift below it, so the
// list costs each lane one entry of registers instead of k.
__device__ __forceinline__ bool better_hit(double ha, uint32_t ia, double hb, uint32_t ib) {
    return ha > hb || (ha == hb && ia < ib);
}

// Top-k of one wavefront kept in LDS (rows of k entries sorted by hyperscore
// desc, id asc), so that no registers stay allocated to it across the scan;
// insertions are rare once the list holds good hits.  Lane j < k handles
// entry j.  Every call is made by all 64 lanes of the wavefront.
template <typename C>
struct WaveTopK {
    double* h;
    uint32_t* id;
    unsigned long long* c;
    __device__ void init(uint32_t k) {
        const uint32_t lane = threadIdx.x & 63u;
        if (lane < k) { h[lane] = -INFINITY; id[lane] = 0xFFFFFFFFu; c[lane] = 0; }
    }
    // Insert a wave-uniform candidate.
    __device__ void insert(double xh, uint32_t xid, C xc, uint32_t k) {
        const uint32_t lane = threadIdx.x & 63u;
        const bool in = lane < k;
        const double hj = in ? h[lane] : 0.0;
        const uint32_t ij = in ? id[lane] : 0u;
        const unsigned long long m = __ballot(in && better_hit(xh, xid, hj, ij));
        if (m == 0) return;
        const uint32_t p = (uint32_t)__ffsll((long long)m) - 1u;
        const bool shift = in && lane > p;
        const double ph = shift ? h[lane - 1] : 0.0;
        const uint32_t pi = shift ? id[lane - 1] : 0u;
        const unsigned long long pc = shift ? c[lane - 1] : 0ull;
        if (shift) { h[lane] = ph; id[lane] = pi; c[lane] = pc; }
        if (lane == p) { h[lane] = xh; id[lane] = xid; c[lane] = (unsigned long long)xc; }
    }
    // Insert every flagged lane's candidate that beats the current k-th best.
    __device__ void insert_lanes(bool flag, double ch, uint32_t cid, C cc, uint32_t k) {
        const double kh = h[k - 1];
        const uint32_t kid = id[k - 1];
        unsigned long long m = __ballot(flag && better_hit(ch, cid, kh, kid));
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            insert(__shfl(ch, l, 64), __shfl(cid, l, 64), (C)__shfl((unsigned long long)cc, l, 64), k);
        }
    }
};

// ---------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(void* p, uint32_t value, uint64_t count, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    uint64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, (uint32_t*)p, value, count);
    return hipGetLastError();
}

__global__ void k_set_header(BatchHdr* hdr, unsigned long long n, unsigned long long nnz) {
    if (threadIdx.x == 0) { hdr->n = n; hdr->nnz = nnz; }
}

hipError_t launch_set_header(BatchHdr* hdr, uint64_t n, uint64_t nnz, hipStream_t stream) {
    hipLaunchKernelGGL(k_set_header, dim3(1), dim3(64), 0, stream, hdr, (unsigned long long)n,
                       (unsigned long long)nnz);
    return hipGetLastError();
}

__global__ void k_fill_per_spectrum(uint32_t* p, uint32_t v, uint64_t per, const BatchHdr* hdr) {
    const uint64_t n = hdr->n * per;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_per_spectrum(void* p, uint32_t value, uint64_t per, uint64_t cap_count, const BatchHdr* hdr,
                                    hipStream_t stream) {
    if (cap_count == 0) return hipSuccess;
    uint64_t blocks = (cap_count + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_per_spectrum, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, (uint32_t*)p, value,
                       per, hdr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// prep: one workgroup per spectrum
// ---------------------------------------------------------------------------

// First index i in [0, n) with mass[i] >= v (upper = false) or mass[i] > v
// (upper = true), n if none: a 64-ary search by one wavefront.  Each round the
// 64 lanes probe evenly spaced positions of the remaining range [a, b) and the
// ballot of "still below" narrows it about 64-fold, so a few dependent loads
// replace the ~22 of a binary search.  Call with the whole wavefront active.
__device__ uint64_t wave_bound(const int64_t* mass, uint64_t n, int64_t v, bool upper) {
    const uint64_t lane = threadIdx.x & 63u;
    uint64_t a = 0, b = n;
    while (a < b) {
        const uint64_t step = (b - a + 63) / 64;
        const uint64_t i = a + (lane + 1) * step - 1;
        bool below = false;
        if (i < b) {
            const int64_t m = mass[i];
            below = upper ? (m <= v) : (m < v);
        }
        const uint64_t c = (uint64_t)__popcll(__ballot(below));
        const uint64_t na = a + c * step;
        if (step == 1) return na;                       // every position was probed
        const uint64_t cap = a + (c + 1) * step - 1;    // probe c failed (or lies beyond b)
        a = na;
        b = cap < b ? cap : b;
    }
    return a;
}

struct PrepArgs {
    DevIndex ix;
    DevSpectra sp;
    KParams kp;
    Work w;
};

// Peaks a spectrum may have for k_prep to stage them in LDS; larger spectra are
// read from global memory.  Small enough that five workgroups fit a CU.
constexpr uint32_t kPrepLdsPeaks = 1024;

// Ranking key of a peak: intensity bits over inverted m/z bits.  For finite
// m/z > 0 and intensity >= 0 (-0 taken as +0) a larger key is a more intense
// peak, or an equally intense one at lower m/z; equal keys are equal peaks.
__device__ __forceinline__ unsigned long long peak_key(float mz, float in) {
    const uint32_t vb = in == 0.0f ? 0u : __float_as_uint(in);
    return ((unsigned long long)vb << 32) | (uint32_t)~__float_as_uint(mz);
}

__global__ __launch_bounds__(kBlock) void k_prep(PrepArgs A) {
    __shared__ unsigned long long s_key[kPrepLdsPeaks];
    __shared__ __align__(16) uint32_t s_ent[PS_MAX_TOP_PEAKS * (PS_MAX_CHARGE - 1)];
    __shared__ uint32_t s_flag, s_imax_bits, s_mult, s_alive;
    __shared__ unsigned long long s_red[kBlock / 64];
    __shared__ uint64_t s_win[2];
    const uint32_t tid = threadIdx.x;
    const KParams& kp = A.kp;

    const uint64_t n_batch = A.sp.hdr->n, nnz_batch = A.sp.hdr->nnz;
    for (uint64_t s = blockIdx.x; s < n_batch; s += gridDim.x) {
        const uint64_t p0 = A.sp.peak_off[s], p1 = A.sp.peak_off[s + 1];
        const int z = A.sp.charge[s];
        const double prec = A.sp.prec[s];
        // filter_1: ids with |M - M_q| <= dM  ->  [lo, hi), searched by wavefronts 0 and 1
        // while the others start on the peaks
        const bool prec_ok = z >= 1 && z <= (int)kp.max_charge && prec > 0.0 && prec <= 1e6;
        const int64_t mq = prec_ok ? (int64_t)z * (round_half_up_pos(prec * 1e6) - kProtonUda) : -1;
        const int64_t dm = mq < 0 ? 0 : kp.window_is_ppm ? (mq * kp.window) / 1000000 : kp.window;
        if ((tid >> 6) < 2) {
            const bool hi_side = (tid >> 6) == 1;
            const uint64_t r = mq < 0 ? 0 : wave_bound(A.ix.mass, A.ix.n_pep, hi_side ? mq + dm : mq - dm, hi_side);
            if ((tid & 63u) == 0) s_win[hi_side ? 1 : 0] = r;
        }
        if (tid == 0) {
            uint32_t bad = 0;
            if (!(p1 >= p0) || p1 - p0 > PS_MAX_PEAKS_IN || p1 > nnz_batch) bad = 1;
            if (z < 1 || z > (int)kp.max_charge) bad = 1;
            if (!(prec > 0.0) || !(prec <= 1e6)) bad = 1;   // also rejects NaN
            s_flag = bad;
            s_imax_bits = 0;
            s_mult = 0;
            s_alive = 0;
        }
        __syncthreads();
        const uint32_t np = s_flag ? 0u : (uint32_t)(p1 - p0);
        for (uint32_t i = tid; i < np; i += kBlock) {
            float m = A.sp.mz[p0 + i], v = A.sp.inten[p0 + i];
            if (np <= kPrepLdsPeaks) s_key[i] = peak_key(m, v);
            if (!(m > 0.0f) || !(m <= 3.0e38f) || !(v >= 0.0f) || !(v <= 3.0e38f)) atomicOr(&s_flag, 1u);
            // ordered like floats for v >= 0; the sign bit is cleared so that -0 counts as +0
            else atomicMax(&s_imax_bits, __float_as_uint(v) & 0x7FFFFFFFu);
        }
        __syncthreads();
        // the peaks: staged in LDS, or read where they are when there are more
        const bool lds = np <= kPrepLdsPeaks;
        const float* gmz = A.sp.mz + p0;
        const float* gin = A.sp.inten + p0;
        auto key_at = [&](uint32_t i) { return lds ? s_key[i] : peak_key(gmz[i], gin[i]); };
        auto mz_at = [&](uint32_t i) { return lds ? __uint_as_float(~(uint32_t)s_key[i]) : gmz[i]; };
        auto in_at = [&](uint32_t i) { return lds ? __uint_as_float((uint32_t)(s_key[i] >> 32)) : gin[i]; };
        const bool bad = s_flag != 0;
        const float imax = __uint_as_float(s_imax_bits);
        const uint32_t cmax = z > 2 ? (uint32_t)(z - 1) : 1u;
        // noise clearing: peaks with I * 1000 < Imax * p (exact in fp64) are dropped.  They
        // are weaker than every peak that stays, so the ranks below are unchanged; only
        // the number kept is limited by the survivors.
        uint32_t alive = np;
        if (kp.noise_permille) {
            uint32_t mine = 0;
            for (uint32_t i = tid; i < np; i += kBlock)
                mine += (double)in_at(i) * 1000.0 >= (double)imax * (double)kp.noise_permille ? 1u : 0u;
            if (mine) atomicAdd(&s_alive, mine);
            __syncthreads();
            alive = s_alive;
        }
        const uint32_t keep = min(alive, kp.top_peaks);
        const uint32_t n_ent = bad ? 0u : keep * cmax;
        uint32_t* gent = A.w.entries + s * (uint64_t)kp.ent_stride;
        // top-B by (intensity desc, m/z asc, input order asc): rank = number of better peaks.
        // When every peak is kept, any order of the entries gives the same search, so a
        // peak's entries go at its input position.
        if (!bad) {
            const bool all_kept = keep == np;
            for (uint32_t i = tid; i < np; i += kBlock) {
                const float mi = mz_at(i), vi = in_at(i);
                const unsigned long long ki = key_at(i);
                uint32_t rank = all_kept ? i : 0u;
                if (all_kept) {
                } else if (lds) {
                    for (uint32_t j = 0; j < np; ++j) {
                        const unsigned long long kj = s_key[j];
                        rank += kj > ki || (kj == ki && j < i);
                    }
                } else {
                    for (uint32_t j = 0; j < np; ++j) {
                        const unsigned long long kj = peak_key(gmz[j], gin[j]);
                        rank += kj > ki || (kj == ki && j < i);
                    }
                }
                if (rank >= keep) continue;
                // integer intensity q in [1, 100] relative to the most intense peak
                uint32_t q = 1;
                if (imax > 0.0f && kp.intensity == PS_INTENSITY_SQRT) {
                    // the largest k with (k - 1/2)^2 <= 10^4 I / Imax; the comparisons are exact
                    const double t = ((double)vi / (double)imax) * 10000.0;
                    int k = (int)(sqrt(t) + 0.5);
                    k = k < 1 ? 1 : (k > 100 ? 100 : k);
                    while (k < 100 && ((double)k + 0.5) * ((double)k + 0.5) <= t) ++k;
                    while (k > 1 && ((double)k - 0.5) * ((double)k - 0.5) > t) --k;
                    q = (uint32_t)k;
                } else if (imax > 0.0f) {
                    double t = (double)vi / (double)imax;
                    t = t * 100.0;
                    t = t + 0.5;
                    t = floor(t);
                    q = t < 1.0 ? 1u : (t > 100.0 ? 100u : (uint32_t)t);
                }
                const double x = (double)mi * 1e6;            // exact: float32 * 10^6 fits in fp64
                // beyond 2^40 uDa no fragment bin exists: such a peak matches nothing
                const int64_t mz_uda = x < 1099511627776.0 ? round_half_up_pos(x) : (1ll << 40);
                for (uint32_t c = 1; c <= cmax; ++c) {
                    // singly charged equivalent of a fragment at charge c
                    const int64_t m1 = (int64_t)c * mz_uda - (int64_t)(c - 1) * kProtonUda;
                    uint32_t e = kEntryInvalid;
                    if (m1 >= 0 && mz_uda < (1ll << 40)) {
                        const int64_t b = (m1 + kBinWidth / 2) / kBinWidth;
                        if (b < (1ll << 24)) e = ((uint32_t)b << 8) | q;
                    }
                    s_ent[rank * cmax + (c - 1)] = e;
                    gent[rank * cmax + (c - 1)] = e;
                }
            }
        }
        __syncthreads();
        // counter-width bound: M = most entries within one 2T+1-bin span
        uint32_t sumq = 0, valid = 0;
        const uint32_t span = 2u * (uint32_t)kp.tol;
        for (uint32_t i = tid; i < n_ent; i += kBlock) {
            const uint32_t ei = s_ent[i];
            if (ei == kEntryInvalid) continue;
            ++valid;
            sumq += ei & 0xFFu;
            const uint32_t bi = ei >> 8;
            // entries with a bin in [bi, bi + span]: the unsigned difference wraps
            // for bins below bi; four entries per LDS read
            auto near = [&](uint32_t ej) { return (uint32_t)(ej != kEntryInvalid && (ej >> 8) - bi <= span); };
            uint32_t m = 0, j = 0;
            for (; j + 4u <= n_ent; j += 4u) {
                const uint4 e = *(const uint4*)&s_ent[j];
                m += near(e.x) + near(e.y) + near(e.z) + near(e.w);
            }
            for (; j < n_ent; ++j) m += near(s_ent[j]);
            atomicMax(&s_mult, m);
        }
        const unsigned long long tot = block_sum<unsigned long long>(
            ((unsigned long long)sumq << 32) | valid, s_red);
        if (tid == 0) {
            SpecInfo inf;
            inf.n_ent = n_ent;
            inf.flags = bad ? kFlagInvalid : 0u;
            inf.lo = inf.hi = 0;
            if (!bad) {
                if (mq < 0) {
                    inf.flags = kFlagInvalid;
                } else {
                    inf.lo = (uint32_t)s_win[0];
                    inf.hi = (uint32_t)s_win[1];
                    // worst-case field values for any candidate of this spectrum
                    const uint64_t nvalid = tot & 0xFFFFFFFFull, sq = tot >> 32;
                    const uint64_t width = (uint64_t)(2 * kp.tol + 1) * (uint64_t)kBinWidth;
                    // (each ion series of a terminus adds at most kpe ions per window)
                    const uint64_t kpe = A.ix.min_residue > 0 ? (width - 1) / (uint64_t)A.ix.min_residue + 1 : (1ull << 20);
                    uint64_t nbmax = nvalid * kpe * A.ix.ion_mult;
                    const uint64_t by_len = (uint64_t)(A.ix.max_len > 0 ? A.ix.max_len - 1 : 0) * (uint64_t)s_mult *
                                            A.ix.ion_mult;
                    if (by_len < nbmax) nbmax = by_len;
                    uint64_t smax = sq * (uint64_t)A.ix.ion_series * kpe;
                    if (200ull * nbmax < smax) smax = 200ull * nbmax;
                    if (!(nbmax <= 255 && smax <= 32767)) {
                        inf.flags |= kFlagWide;
                        if (!(nbmax < kLfSize && smax < kLsSize)) inf.flags |= kFlagOverflow;
                        atomicAdd(&A.w.counters[(inf.flags & kFlagOverflow) ? kCtrOverflow : kCtrWide], 1ull);
                    }
                }
            }
            A.w.info[s] = inf;
        }
        __syncthreads();
    }
}

hipError_t launch_prep(const DevIndex& ix, const DevSpectra& sp, const KParams& kp, const Work& w,
                       hipStream_t stream) {
    if (sp.n == 0) return hipSuccess;
    PrepArgs a{ix, sp, kp, w};
    uint64_t grid = sp.n < (1u << 20) ? sp.n : (1u << 20);
    hipLaunchKernelGGL(k_prep, dim3((uint32_t)grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scan: shared-peak counting in LDS tiles + scoring
// ---------------------------------------------------------------------------

struct ScanArgs {
    DevIndex ix;
    DevSpectra sp;
    KParams kp;
    Work w;
    uint32_t tiles_per_item;   // persistent schedule
    uint32_t want_wide;        // which counter width this launch handles
    uint32_t per_item;         // partial lists indexed by work item (persistent schedule)
};

// The scan runs in workgroups of NT = 256 or 512 threads (4 or 8 wavefronts)
// sharing one tile of counters; a tile has at least 16 NT ids, so the filter
// reads whole passes of 16-byte counter groups.
constexpr uint32_t kRounds = 1;       // gather rounds of 64 posting quads a wavefront keeps in flight
constexpr uint32_t kWaveCand = 128;   // candidates each wavefront buffers before scoring (two rounds)
template <uint32_t NT> constexpr uint32_t cand_cap() { return kWaveCand * (NT / 64); }
constexpr uint32_t kMapCap = 4096;    // flat quad positions mapped to slots at a time
constexpr uint32_t kDenseProbes = 4;  // probes of a work item read from dense maps (others are streamed)
constexpr uint32_t kDenseFloor = 2;   // lowest candidate-filter threshold that map probes may leave
// map words: one per 64 quads, plus one for the start bit just past the chunk
constexpr uint32_t kMapWords = kMapCap / 64 + 1;
// s_waitcnt operand (gfx9 encoding): vmcnt(0), expcnt and lgkmcnt left at their maxima
constexpr int kWaitVmem0 = 0x0F70;

template <uint32_t NT>
struct ScanShared {
    uint32_t nact;
    uint32_t ndense, dused;                    // map probes kept; their count bounds claimed
    uint32_t dtab[kMaxDense];                  // the index's dense table
    uint32_t dprobe[kDenseProbes];             // q | bound << 8 of each map probe
    const uint8_t* dmap[kDenseProbes];         // its map
    unsigned long long acc_post, acc_look;     // the item's postings and bin lookups
    unsigned long long acc_dpost, acc_dreads;  // postings counted from maps; map reads
    unsigned long long wsum[NT / 64];
    unsigned long long red[NT / 64];
    double wh[NT / 64][PS_MAX_TOP_K];          // per-wavefront top-k lists
    uint32_t wid[NT / 64][PS_MAX_TOP_K];
    unsigned long long wc[NT / 64][PS_MAX_TOP_K];
    uint32_t head[NT / 64];                    // merge cursors of the final top-k (thread 0)
};

// What the lookup pass finds for one fragment-bin probe with postings in the
// item: its bin, the first quad of the bin's list, its posting run [s0, s1)
// inside the item, the peak's integer intensity and the ends of the run's first
// two tiles (positions inside the bin's list).
struct SlotInit {
    uint32_t bin, qb, s0, s1, q, e0, e1;
};

// A slot with postings in the current tile, by rank among such slots.  Its run
// [cur, end) is read in aligned quads of postings: flat quad position f of its
// range reads quad base + f of the posting array.  qx = q (its peak's
// intensity) | lead << 8 (postings before cur in its first quad) | (tail - 1)
// << 10 (postings of the run in its last quad, 1..4).
struct SegBase {
    uint32_t base, qx;
};

// LDS layout (dynamic):
//   counters (the SlotInit array before the first tile) | SegBase[seg_cap] |
//   map bits [kMapWords] (u64) | range starts [seg_cap] | list quads [seg_cap] |
//   map ranks [kMapCap / 64] | candidate counters | histogram | candidate positions
//
// The map of a chunk of kMapCap flat positions: bit b of mbits[R] is set when
// a slot's range starts at position 64 R + b, and mrank[R] is the rank of the
// slot holding position 64 R, so the slot of any position is one popcount away.
template <typename C, uint32_t NT>
struct ScanLds {
    C* cnt;
    SlotInit* init;
    SegBase* sbase;
    uint32_t* sstart;
    uint32_t* sqb;        // [seg_cap] first quad of each slot's bin list, by slot
    unsigned long long* mbits;
    uint32_t* mrank;
    C* cand_cnt;          // [cand_cap] counters of candidates that passed the filter, kWaveCand per wavefront
    int32_t* hist;
    uint32_t* cand_id;    // [cand_cap] their peptide ids
    __device__ ScanLds(uint8_t* base, uint32_t tile, uint32_t segcap) {
        size_t o = 0;
        cnt = (C*)base;
        init = (SlotInit*)base;
        const size_t head = max((size_t)tile * sizeof(C), (size_t)segcap * sizeof(SlotInit));
        o += (head + 15) & ~(size_t)15;
        sbase = (SegBase*)(base + o); o += (size_t)segcap * sizeof(SegBase);
        mbits = (unsigned long long*)(base + o); o += (size_t)kMapWords * 8;
        sstart = (uint32_t*)(base + o); o += (size_t)segcap * 4;
        sqb = (uint32_t*)(base + o); o += (size_t)segcap * 4;
        mrank = (uint32_t*)(base + o); o += (size_t)(kMapCap / 64) * 4;
        o = (o + 15) & ~(size_t)15;
        cand_cnt = (C*)(base + o); o += (size_t)cand_cap<NT>() * sizeof(C);
        hist = (int32_t*)(base + o); o += (size_t)kHistBins * 4;
        cand_id = (uint32_t*)(base + o);
    }
};

size_t scan_lds_bytes(const KParams& kp, bool wide) {
    const size_t csz = wide ? 8 : 4;
    const size_t cap = (size_t)kWaveCand * (kp.nt / 64);
    const size_t head = std::max((size_t)kp.tile * csz, (size_t)kp.seg_cap * sizeof(SlotInit));
    size_t o = (head + 15) & ~(size_t)15;
    o += (size_t)kp.seg_cap * (sizeof(SegBase) + 8) + (size_t)kMapWords * 8 + (size_t)(kMapCap / 64) * 4;
    o = (o + 15) & ~(size_t)15;
    o += cap * csz;
    o += (size_t)kHistBins * 4;
    o += cap * 4;
    return (o + 15) & ~(size_t)15;
}

// Hyperscore of one candidate that passed the filter: log10(n_b! n_y! S) from
// the fp64 tables (log10 S passed in), plus its histogram bin (width 0.1,
// last bin open).
template <typename C, bool DUMP, uint32_t NT>
__device__ __forceinline__ double score_finish(const ScanArgs& A, ScanLds<C, NT>& L, uint32_t s, uint32_t id, C c,
                                               double ls_sq, uint32_t& scored) {
    const uint32_t nb = Cnt<C>::nb(c), ny = Cnt<C>::ny(c), sq = Cnt<C>::s(c);
    const double h = (A.ix.lf[nb] + A.ix.lf[ny]) + ls_sq;
    const double hb = floor(10.0 * h);
    const int bin = hb >= (double)(kHistBins - 1) ? kHistBins - 1 : (int)hb;
    atomicAdd(&L.hist[bin], 1);
    ++scored;
    if (DUMP) {
        const unsigned long long slot = atomicAdd(&A.w.counters[kCtrDump], 1ull);
        if (slot < A.w.dump_cap) {
            A.w.dump_spec[slot] = s;
            A.w.dump_id[slot] = id;
            A.w.dump_cnt_lo[slot] = (nb & 0xFFFFu) | (ny << 16);
            A.w.dump_cnt_hi[slot] = sq;
        }
    }
    return h;
}

template <typename C, bool DUMP, uint32_t NT>
__device__ __forceinline__ double score_one(const ScanArgs& A, ScanLds<C, NT>& L, uint32_t s, uint32_t id, C c,
                                            uint32_t& scored) {
    return score_finish<C, DUMP, NT>(A, L, s, id, c, A.ix.ls[Cnt<C>::s(c)], scored);
}

// Exclusive prefix sum over the workgroup in thread order; *total gets the sum.
// Contains one barrier; `wsum` must not be in use by another pass.
template <typename T, uint32_t NT>
__device__ __forceinline__ T block_exclusive_scan(T v, T* wsum, T* total) {
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    T x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63u) wsum[wave] = x;
    __syncthreads();
    T before = 0, all = 0;
    for (uint32_t w = 0; w < NT / 64; ++w) {
        const T t = wsum[w];
        before += w < wave ? t : (T)0;
        all += t;
    }
    *total = all;
    return before + x - v;
}

// Inclusive prefix sum over one wavefront: DPP row shifts within each 16-lane
// row, then row broadcasts (each step adds only where the lane condition holds,
// so out-of-row sources never matter).
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false); if ((lane & 15u) >= 1u) x += t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false); if ((lane & 15u) >= 2u) x += t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false); if ((lane & 15u) >= 4u) x += t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false); if ((lane & 15u) >= 8u) x += t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xF, 0xF, false); if ((lane & 31u) >= 16u) x += t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xF, 0xF, false); if (lane >= 32u) x += t;
    return x;
}

// Exclusive prefix sums over the workgroup (thread order) of a count n and of a
// small number e <= U, with their totals.  One barrier; `wsum` must be free.
// A wavefront that is not `active` (wave-uniform) has n = e = 0 in every
// lane and skips its own scan: its wsum entry must already hold 0.
template <uint32_t U, uint32_t NT>
__device__ __forceinline__ void block_scan_counts(bool active, uint32_t n, uint32_t e, unsigned long long* wsum,
                                                  uint32_t* n_ex, uint32_t* e_ex, uint32_t* n_all, uint32_t* e_all) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar selects below
    uint32_t incl = 0, ex = 0, et = 0;
    if (active) {
        incl = wave_inclusive_sum(n);
#pragma unroll
        for (uint32_t b = 0; (1u << b) <= U; ++b) {    // e bit by bit: ballot + mbcnt
            const unsigned long long m = __ballot((e >> b) & 1u);
            ex += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << b;
            et += (uint32_t)__popcll(m) << b;
        }
        const uint32_t ntot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);   // scalar: no lane address
        if (lane == 0) wsum[wave] = ((unsigned long long)et << 32) | ntot;
    }
    __syncthreads();
    // lane w < NT / 64 takes wavefront w's totals; inclusive sums over those
    // lanes (inside the first 16-lane DPP row) give every wavefront its
    // offsets and the totals by lane reads
    const unsigned long long wv = lane < NT / 64 ? wsum[lane] : 0ull;
    uint32_t xn = (uint32_t)wv, xe = (uint32_t)(wv >> 32), t;
    static_assert(NT / 64 <= 8, "one DPP row holds the wavefront totals");
    // row_shr:1, 2, 4 (DPP controls 0x111, 0x112, 0x114)
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)xn, 0x111, 0xF, 0xF, false); if ((lane & 15u) >= 1u) xn += t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)xe, 0x111, 0xF, 0xF, false); if ((lane & 15u) >= 1u) xe += t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)xn, 0x112, 0xF, 0xF, false); if ((lane & 15u) >= 2u) xn += t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)xe, 0x112, 0xF, 0xF, false); if ((lane & 15u) >= 2u) xe += t;
    if constexpr (NT / 64 > 4) {
        t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)xn, 0x114, 0xF, 0xF, false); if ((lane & 15u) >= 4u) xn += t;
        t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)xe, 0x114, 0xF, 0xF, false); if ((lane & 15u) >= 4u) xe += t;
    }
    const uint32_t na = (uint32_t)__builtin_amdgcn_readlane((int)xn, NT / 64 - 1);
    const uint32_t ea = (uint32_t)__builtin_amdgcn_readlane((int)xe, NT / 64 - 1);
    const uint32_t nb = wave ? (uint32_t)__builtin_amdgcn_readlane((int)xn, (int)wave - 1) : 0u;
    const uint32_t eb = wave ? (uint32_t)__builtin_amdgcn_readlane((int)xe, (int)wave - 1) : 0u;
    *n_ex = nb + incl - n;
    *e_ex = eb + ex;
    *n_all = na;
    *e_all = ea;
}

// Enter the slot of rank k, whose range is [a, b), into the map of the chunk
// [c0, c0 + kMapCap): its start bit, and the rank of every 64-position round
// that begins inside it.
// A start exactly at the chunk's end is entered too (word kMapCap / 64): it
// ends the chunk's last slot.
template <typename C, uint32_t NT>
__device__ __forceinline__ void map_slot(const ScanLds<C, NT>& L, uint32_t k, uint32_t a, uint32_t b, uint32_t c0) {
    const uint32_t ce = c0 + kMapCap;
    if (a >= c0 && a <= ce) atomicOr(&L.mbits[(a - c0) >> 6], 1ull << ((a - c0) & 63u));
    if (b <= c0 || a >= ce) return;
    const uint32_t lo = max(a, c0), hi = min(b, ce);
    for (uint32_t r = (lo - c0 + 63u) >> 6; (r << 6) < hi - c0; ++r) L.mrank[r] = k;
}

// Gather state of one wavefront in the current chunk [c0, fe) of flat quad
// positions.  The chunk is dealt out in batches of kRounds x 64 positions,
// batch j to wavefront j mod (NT / 64), so a tile with few postings occupies
// few wavefronts and none of them runs an empty batch; `next` is the start
// of this wavefront's next batch.  `live` says whether the batch in flight
// holds any position (wave-uniform), and p / mq hold its loaded postings.
struct Gather {
    uint32_t c0, fe, next;             // quad positions
    uint32_t live;
    uint4 p[kRounds];
    uint32_t mq[(kRounds + 1) / 2];    // round r in half r % 2: elements of the run (bits 0-3) | q << 4
};

// Map flat quad positions [g.next, g.next + 64 * kRounds) of this wavefront
// to slots through the chunk map and issue their posting loads (16 aligned
// bytes per lane).  A round is 64 aligned positions, so its map word and round
// rank are broadcast reads.  A quad is the first of its slot when its own
// start bit is set and the last when the next position's is (the bit past
// the chunk, or the end marker after the last slot): only there do postings
// outside the run share the quad.
//
// Every lane issues its loads (a lane past the chunk reads quad 0 and keeps
// no element of it), so a batch is always kRounds loads in straight-line code
// and the compiler can wait for an older batch while a newer one is in flight.
// LIVE: the caller knows the wavefront has a batch left.
template <typename C, uint32_t NT, bool LIVE = false>
__device__ __forceinline__ void gather_issue(const DevIndex& ix, const ScanLds<C, NT>& L, Gather& g) {
    const uint32_t lane = threadIdx.x & 63u;
    const unsigned long long below = (2ull << lane) - 2ull;   // positions 1..lane of a round
#pragma unroll
    for (uint32_t r = 0; r < (kRounds + 1) / 2; ++r) g.mq[r] = 0;
    g.live = LIVE || g.next < g.fe;
    if (!LIVE && !g.live) return;                      // wave-uniform: no batch left for this wavefront
#pragma unroll
    for (uint32_t r = 0; r < kRounds; ++r) {
        const uint32_t f = g.next + 64u * r + lane;
        const bool valid = f < g.fe;
        const uint32_t R = min((g.next - g.c0) / 64u + r, kMapCap / 64u - 1u);   // clamped: rounds past fe
        const unsigned long long bits = L.mbits[R];
        const unsigned long long after = L.mbits[R + 1];
        const uint32_t k = L.mrank[R] + (uint32_t)__popcll(bits & below);
        const SegBase sb = L.sbase[valid ? k : 0u];
        g.p[r] = ((const uint4*)ix.post)[valid ? sb.base + f : 0u];
        const bool first = (bits >> lane) & 1ull;
        const bool last = (lane < 63u ? (bits >> (lane + 1u)) : after) & 1ull;
        const uint32_t lead = first ? (sb.qx >> 8) & 3u : 0u;
        const uint32_t keep = last ? ((sb.qx >> 10) & 3u) + 1u : 4u;
        const uint32_t m4 = valid ? (0xFu << lead) & (0xFu >> (4u - keep)) : 0u;
        g.mq[r / 2] |= (m4 | (sb.qx & 0xFFu) << 4) << (16u * (r % 2u));
    }
    g.next += NT * kRounds;                            // this wavefront's next batch
}

template <typename C, uint32_t NT>
__device__ __forceinline__ void gather_consume(const ScanLds<C, NT>& L, const Gather& g, uint32_t tsh) {
    if (!g.live) return;                               // wave-uniform
#pragma unroll
    for (uint32_t r = 0; r < kRounds; ++r) {
        const uint32_t w = g.mq[r / 2] >> (16u * (r % 2u));
        if (w & 0xFu) {
            const uint32_t q = (w >> 4) & 0xFFu;
            const uint32_t e4[4] = {g.p[r].x, g.p[r].y, g.p[r].z, g.p[r].w};
            // Every element is added without a branch: one outside the run (a
            // neighbouring run's posting or list padding in the same quad) adds 0
            // to the counter its bits select.  Tiles are aligned to their size:
            // the counter is the id modulo the tile.
#pragma unroll
            for (uint32_t e = 0; e < 4; ++e) {
                const uint32_t p = e4[e];
                const C keep = (C)0 - (C)((w >> e) & 1u);          // all ones inside the run
                atomicAdd(&L.cnt[__builtin_amdgcn_ubfe(p, 1u, tsh)], Cnt<C>::inc(p & 1u, q) & keep);
            }
        }
    }
}

// One work item: spectrum s, candidate ids [ida, idb).  Writes the item's top
// hits to `out` (top_k entries) and adds its histogram and counts to the
// spectrum's global accumulators.
//
// Lookup (filter_2): every (entry, bin offset) probe gives the bin's posting
// run inside [ida, idb) from the tile directory (a search inside one
// directory block only where ida or idb is not on a block edge).  Runs that
// are not empty become probe slots, held in registers by their owner threads.
//
// Tiles: candidates [t * tile, (t + 1) * tile) share one LDS counter array.
// The directory gives every run's tile boundaries directly, so the postings
// of tile t + 1 are mapped and loaded while tile t is filtered and scored,
// and the boundaries of tile t + 2 are loaded one tile earlier still.
template <typename C, bool DUMP, uint32_t U, uint32_t NT>
__device__ void scan_item(const ScanArgs& A, ScanShared<NT>& sh, ScanLds<C, NT>& L, uint32_t s, uint32_t ida,
                          uint32_t idb, ps_hit* out) {
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar addressing
    const KParams& kp = A.kp;
    const DevIndex& ix = A.ix;
    const uint32_t n_ent = A.w.info[s].n_ent;
    const uint32_t* ent = A.w.entries + (uint64_t)s * kp.ent_stride;
    // probes per entry: the 2T+1 bins around it, or its one merged list
    const int T = ix.merge_tol ? 0 : kp.tol;
    const uint32_t width = (uint32_t)(2 * T + 1);
    const uint32_t gsh = ix.dir_shift, tsh = kp.tile_shift;
    const uint64_t stride = ix.dir_stride;
    const uint32_t m = kp.tile >> gsh;                 // directory entries per tile
    const uint32_t t0 = ida >> tsh, t_last = (idb - 1) >> tsh;

    if (tid == 0) {
        sh.nact = 0; sh.ndense = 0; sh.dused = 0;
        sh.acc_post = 0; sh.acc_look = 0; sh.acc_dpost = 0; sh.acc_dreads = 0;
    }
    for (uint32_t i = tid; i < (uint32_t)kHistBins; i += NT) L.hist[i] = 0;
    if (tid < ix.n_dense) sh.dtab[tid] = ix.dense_tab[tid];
    __syncthreads();

    // end of tile u's part of a run that ends at s1
    auto tile_end = [&](const uint32_t* row, uint32_t u, uint32_t s1) -> uint32_t {
        const uint64_t edge = (uint64_t)(u + 1) << tsh;
        return edge >= idb ? s1 : min(s1, row[edge >> gsh]);
    };

    unsigned long long lookups = 0, postings = 0, dpost = 0;
    const uint32_t npairs = n_ent * width;
    // Map probes lower the filter's threshold by the most they can add to one
    // id's count; they are taken only while it stays at kDenseFloor or more.
    const uint32_t dbudget = kp.min_shared >= kDenseFloor ? kp.min_shared - kDenseFloor : 0u;
    const uint32_t gmask = (1u << gsh) - 1u;
    for (uint32_t k = tid; k < npairs; k += NT) {
        const uint32_t e = ent[k / width];
        if (e == kEntryInvalid) continue;
        const int64_t bin = (int64_t)(e >> 8) + (int64_t)(k % width) - T;
        if (bin < 0 || bin >= (int64_t)ix.n_bins) continue;
        ++lookups;
        const uint32_t* row = ix.dir + (uint64_t)bin * stride;
        const uint32_t ka = ida >> gsh, kb = idb >> gsh;
        const uint32_t qb = ix.bin_q[bin];
        const uint32_t* list = ix.post + 4ull * qb;
        const uint32_t s0 = (ida & gmask) ? lower_bound_u32(list, row[ka], row[ka + 1], ida << 1) : row[ka];
        const uint32_t s1 = (idb & gmask) ? lower_bound_u32(list, row[kb], row[kb + 1], idb << 1) : row[kb];
        if (s1 <= s0) continue;
        postings += s1 - s0;
        if (ix.n_dense && dbudget) {
            uint32_t hit = 0;                           // the list's table entry (never 0)
            for (uint32_t j = 0; j < ix.n_dense; ++j) {
                const uint32_t t = sh.dtab[j];
                if ((t & 0xFFFFFFu) == (uint32_t)bin) hit = t;
            }
            const uint32_t mc = (hit >> 24) & 3u;
            if (hit && atomicAdd(&sh.dused, mc) + mc <= dbudget) {
                const uint32_t j = atomicAdd(&sh.ndense, 1u);
                if (j < kDenseProbes) {
                    sh.dprobe[j] = (e & 0xFFu) | mc << 8;
                    sh.dmap[j] = ix.dense_maps + (uint64_t)(hit >> 28) * ix.dense_stride;
                    dpost += s1 - s0;
                    continue;
                }
            }
        }
        const uint32_t slot = atomicAdd(&sh.nact, 1u);
        SlotInit si;
        si.bin = (uint32_t)bin;
        si.qb = qb;
        si.s0 = s0;
        si.s1 = s1;
        si.q = e & 0xFFu;
        si.e0 = tile_end(row, t0, s1);
        si.e1 = t0 < t_last ? tile_end(row, t0 + 1, s1) : s1;
        L.init[slot] = si;
    }
    // the item's postings and lookups: a wavefront sum, added in LDS
    for (int o = 32; o > 0; o >>= 1) {
        postings += __shfl_down(postings, o, 64);
        lookups += __shfl_down(lookups, o, 64);
        dpost += __shfl_down(dpost, o, 64);
    }
    if (lane == 0) {
        if (postings) atomicAdd(&sh.acc_post, postings);
        if (lookups) atomicAdd(&sh.acc_look, lookups);
        if (dpost) atomicAdd(&sh.acc_dpost, dpost);
    }
    __syncthreads();
    const uint32_t nact = sh.nact;
    // what the map probes can add to one id's count at most
    uint32_t dsum = 0;
    for (uint32_t j = 0; j < min(sh.ndense, kDenseProbes); ++j) dsum += sh.dprobe[j] >> 8;
    dsum = __builtin_amdgcn_readfirstlane(dsum);
    // slots [tid * us, tid * us + us) belong to this thread
    const uint32_t us = nact > NT ? (nact + NT - 1) / NT : 1u;
    // wavefronts holding no slot skip the per-tile scan; their totals are 0
    const bool owner = wave * 64u * us < nact;
    if (!owner && lane == 0) sh.wsum[wave] = 0ull;
    // Each slot also holds the aligned quad of its directory row that contains
    // the entry for the end of tile t + 2 (needed when moving to tile t + 1):
    // a quad serves four tiles (one tile = m entries), and the next quad is
    // loaded one tile before its first use.
    auto needs_dir = [&](uint32_t u) { return ((uint64_t)(u + 1) << tsh) < (uint64_t)idb; };   // end(u) < s1?
    auto quad_at = [&](uint32_t bin, uint32_t idx) {
        asm volatile("" : "+v"(bin));                  // keep the row address inside the loop (no hoisted pair to spill)
        return *(const uint4*)(ix.dir + (uint64_t)bin * stride + (idx & ~3u));
    };
    uint32_t o_bq[U], o_s1[U], o_cur[U], o_end[U], o_nxt[U];   // o_bq = bin | q << 24
    uint4 o_quad[U];
    const bool quad0 = t0 + 2 <= t_last && needs_dir(t0 + 2);
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
        const uint32_t j = tid * us + u;
        o_bq[u] = 0; o_s1[u] = 0; o_cur[u] = 0; o_end[u] = 0; o_nxt[u] = 0;
        o_quad[u] = make_uint4(0u, 0u, 0u, 0u);
        if (u < us && j < nact) {
            const SlotInit si = L.init[j];
            L.sqb[j] = si.qb;
            o_bq[u] = si.bin | (si.q << 24); o_s1[u] = si.s1;
            o_cur[u] = si.s0; o_end[u] = si.e0; o_nxt[u] = si.e1;
            if (quad0) o_quad[u] = quad_at(si.bin, (t0 + 3) * m);
        }
    }
    __syncthreads();                                   // SlotInit area becomes the counters

    WaveTopK<C> top{sh.wh[wave], sh.wid[wave], sh.wc[wave]};
    top.init(kp.top_k);
    const uint32_t kk = kp.top_k;
    // filter threshold on counter keys: lowered by what the map probes can add
    // (the exact test follows when candidates are scored)
    const uint32_t kkey = Cnt<C>::key_min(kp.min_shared - dsum);
    uint32_t scored = 0;
    Gather g;
    uint32_t ptot = 0;

    // flat map of tile t's postings from the owned slots' [cur, end) runs, then
    // this wavefront's first gather batch
    uint32_t nne = 0;                                   // slots with postings in the prepared tile

    // the chunk [c0, c0 + kMapCap) of a tile with `total` flat positions, and
    // this wavefront's first batch in it
    auto share = [&](uint32_t c0, uint32_t total) {
        g.c0 = c0;
        g.fe = c0 + min(kMapCap, total - c0);
        g.next = c0 + wave * (64u * kRounds);
    };

    // ranks, flat ranges and the map of the first chunk of the tile whose
    // slots hold [o_cur, o_end), then this wavefront's first gather batch
    // quads of postings a run [cur, end) covers (0 when empty)
    auto quads = [](uint32_t cur, uint32_t end) { return end > cur ? ((cur & 3u) + (end - cur) + 3u) >> 2 : 0u; };
    auto prepare = [&]() {
        for (uint32_t i = tid; i < kMapWords; i += NT) L.mbits[i] = 0ull;
        uint32_t mine = 0, mine_ne = 0;
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {                 // unowned slots are 0 - 0
            const uint32_t n = quads(o_cur[u], o_end[u]);
            mine += n;
            mine_ne += n != 0u;
        }
        uint32_t run, rank, total_n, total_ne;
        block_scan_counts<U, NT>(owner, mine, mine_ne, sh.wsum, &run, &rank, &total_n, &total_ne);
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t n = quads(o_cur[u], o_end[u]);
            if (n) {
                const uint32_t a = o_cur[u] & ~3u;      // the run's first aligned quad (lists start on quads)
                SegBase sb;
                sb.base = L.sqb[tid * us + u] + (a >> 2) - run;   // modulo 2^32: base + f is the quad
                // the intensity is taken from o_bq here, every tile: the empty asm
                // keeps the compiler from hoisting o_bq >> 24 out of the tile loop
                // as a second live register (which it then spills)
                uint32_t bq = o_bq[u];
                asm volatile("" : "+v"(bq));
                sb.qx = (bq >> 24) | (o_cur[u] & 3u) << 8 | (o_end[u] - a - 4u * (n - 1u) - 1u) << 10;
                L.sbase[rank] = sb;
                L.sstart[rank] = run;
                map_slot<C, NT>(L, rank, run, run + n, 0u);
                run += n;
                ++rank;
            }
        }
        ptot = total_n;
        nne = total_ne;
        if (tid == 0 && total_n <= kMapCap) atomicOr(&L.mbits[total_n >> 6], 1ull << (total_n & 63u));   // end marker
        __syncthreads();
        share(0u, ptot);
        gather_issue<C, NT>(ix, L, g);
    };

    // Consume the batch in g, and any further batches of this wavefront in
    // the chunk: each is requested before the one before it is consumed, so
    // its loads are in flight meanwhile.
    auto drain = [&]() {
        while (g.next < g.fe) {
            Gather h = g;
            gather_issue<C, NT, true>(ix, L, h);
            gather_consume<C, NT>(L, g, tsh);
            g = h;
        }
        gather_consume<C, NT>(L, g, tsh);
    };

    if (nact > 0) {
        for (uint32_t i = tid; i < kp.tile; i += NT) L.cnt[i] = (C)0;
        prepare();
    }
    // The directory quad loaded in one tile is first used right after the next
    // tile's posting batch is consumed, where the wavefront waits for its loads
    // anyway.  Each wavefront buffers its own candidates (kWaveCand slots from wbuf) and
    // scores them itself, so the filter needs no shared counter or barrier.
    const uint32_t wbuf = wave * kWaveCand;
    // Candidates collect over tiles and are scored in full rounds of 64 while
    // the item runs (the rest of a round moves to the front of the buffer), and
    // all that is left at the end of the item.
    uint32_t wn = 0;                                    // wave-uniform: candidates buffered
    // With map probes, a buffered candidate first adds its bits from each map
    // (C-terminal bit id % 4, N-terminal bit 4 + id % 4 of byte id / 4) and is
    // scored only if its exact count reaches min_shared.
    auto score_buffer = [&](bool full_rounds) {
        const uint32_t end = full_rounds ? wn & ~63u : wn;
        for (uint32_t base = 0; base < end; base += 64u) {
            const uint32_t j = base + lane;
            bool ok = j < wn;
            C c = ok ? L.cand_cnt[wbuf + j] : (C)0;
            const uint32_t id = ok ? L.cand_id[wbuf + j] : 0u;
            const uint32_t nd = __builtin_amdgcn_readfirstlane(min(sh.ndense, kDenseProbes));
            if (nd) {                                   // uniform
#pragma unroll 1
                for (uint32_t p = 0; p < nd; ++p) {
                    // the map address, made uniform (readfirstlane returns int:
                    // each half goes through uint32_t so that none is sign-extended)
                    const uint64_t a = (uint64_t)sh.dmap[p];
                    const uint32_t a_lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a);
                    const uint32_t a_hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
                    const uint8_t* mp = (const uint8_t*)((uint64_t)a_hi << 32 | (uint64_t)a_lo);
                    const uint32_t q = __builtin_amdgcn_readfirstlane(sh.dprobe[p] & 0xFFu);
                    const uint32_t x = ok ? (uint32_t)mp[id >> 2] >> (id & 3u) : 0u;
                    c += ((x & 1u) ? Cnt<C>::inc(1u, q) : (C)0) + ((x & 16u) ? Cnt<C>::inc(0u, q) : (C)0);
                }
                const unsigned long long m = __ballot(ok);
                if (lane == 0) atomicAdd(&sh.acc_dreads, (unsigned long long)nd * __popcll(m));
                ok = ok && Cnt<C>::key(c) >= Cnt<C>::key_min(kp.min_shared);
            }
            const double h = ok ? score_one<C, DUMP, NT>(A, L, s, id, c, scored) : -INFINITY;
            top.insert_lanes(ok, h, id, c, kk);
        }
        // what is left of a partial round moves to the front (one wavefront:
        // every lane reads before it writes, and the ranges do not overlap)
        const uint32_t rest = wn - end;
        const bool mv = lane < rest;
        const C rc = mv ? L.cand_cnt[wbuf + end + lane] : (C)0;
        const uint32_t rid = mv ? L.cand_id[wbuf + end + lane] : 0u;
        if (mv) { L.cand_cnt[wbuf + lane] = rc; L.cand_id[wbuf + lane] = rid; }
        wn = rest;
    };
    const uint32_t t_end = nact > 0 ? t_last + 1 : t0;
    for (uint32_t t = t0; t < t_end; ++t) {
        const uint32_t tb = t << tsh;
        // counters of tile t: the batch loaded last, then any further batches,
        // then any further chunks
        drain();
        const uint32_t p_t = ptot;
        for (uint32_t c0 = kMapCap; c0 < p_t; c0 += kMapCap) {
            __syncthreads();                            // every wavefront is done with the last map
            for (uint32_t i = tid; i < kMapWords; i += NT) L.mbits[i] = 0ull;
            __syncthreads();
            for (uint32_t k = tid; k < nne; k += NT)
                map_slot<C, NT>(L, k, L.sstart[k], k + 1 < nne ? L.sstart[k + 1] : p_t, c0);
            if (tid == 0 && p_t - c0 <= kMapCap) atomicOr(&L.mbits[(p_t - c0) >> 6], 1ull << ((p_t - c0) & 63u));
            __syncthreads();
            share(c0, p_t);
            gather_issue<C, NT>(ix, L, g);
            drain();
        }
        // end of tile t + 2 from the quad holding directory entry (t + 3) m
        const bool use = t + 2 <= t_last && needs_dir(t + 2);
        const uint32_t idx = (t + 3) * m;
        uint32_t nxt2[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint4 qd = o_quad[u];
            const uint32_t e = (idx & 3u) == 0u ? qd.x : (idx & 3u) == 1u ? qd.y : (idx & 3u) == 2u ? qd.z : qd.w;
            nxt2[u] = use ? min(o_s1[u], e) : o_s1[u];
        }
        // Everything loaded so far has arrived (the batch above needed it).  Say
        // so explicitly: the compiler's load scoreboard then starts clean, so
        // registers reused below never wait for the loads issued next.
        __builtin_amdgcn_s_waitcnt(kWaitVmem0);
        __syncthreads();
        if (t < t_last) {
            // Slots move to tile t + 1 (the quad for the next tile's boundary is
            // requested when it differs from the one just used), and tile t + 1
            // is mapped and its first posting batch issued before tile t is
            // filtered, so the filter hides the load latency.  The map is free:
            // every wavefront is past the barrier above.
            const bool fetch = t + 3 <= t_last && needs_dir(t + 3) && (((t + 4) * m) >> 2) != (idx >> 2);
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                o_cur[u] = o_end[u];
                o_end[u] = o_nxt[u];
                o_nxt[u] = nxt2[u];
                const uint32_t j = tid * us + u;
                if (fetch && u < us && j < nact) o_quad[u] = quad_at(o_bq[u] & 0xFFFFFFu, (t + 4) * m);
            }
            prepare();
        }
        // candidate filter: counters are read and cleared four (narrow) or two
        // (wide) at a time; candidates with at least k_min shared peaks are
        // buffered for scoring
        if (p_t != 0) {                                 // else the counters are all 0
            constexpr uint32_t kPer = 16 / sizeof(C);
            const uint32_t nvec = kp.tile / kPer;
            uint4* cv = (uint4*)L.cnt;
            // nvec is a multiple of 4 NT: four steps per pass, at fixed offsets
            for (uint32_t base0 = wave * 64u; base0 < nvec; base0 += 4u * NT) {
                uint4* cp = cv + base0 + lane;
#pragma unroll
            for (uint32_t step = 0; step < 4u; ++step) {
                const uint4 v = cp[step * NT];
                cp[step * NT] = make_uint4(0u, 0u, 0u, 0u);
                C c[kPer];
                if constexpr (kPer == 4) {
                    c[0] = (C)v.x; c[1] = (C)v.y; c[2] = (C)v.z; c[3] = (C)v.w;
                } else {
                    c[0] = (C)(((unsigned long long)v.y << 32) | v.x);
                    c[1] = (C)(((unsigned long long)v.w << 32) | v.z);
                }
                // most counter groups hold no candidate: one test for the group first
                uint32_t key[kPer];
                uint32_t top = 0;
#pragma unroll
                for (uint32_t e = 0; e < kPer; ++e) { key[e] = Cnt<C>::key(c[e]); top = max(top, key[e]); }
                if (__ballot(top >= kkey) == 0ull) continue;   // wave-uniform
                const uint32_t i = base0 + step * NT + lane;
#pragma unroll
                for (uint32_t e = 0; e < kPer; ++e) {
                    const bool pass = key[e] >= kkey;
                    const unsigned long long msk = __ballot(pass);
                    if (msk == 0) continue;             // wave-uniform
                    if (wn > kWaveCand - 64u) score_buffer(true);   // room for a whole wavefront
                    const uint32_t off = wn + __builtin_amdgcn_mbcnt_hi((uint32_t)(msk >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)msk, 0u));
                    if (pass) {
                        L.cand_id[wbuf + off] = tb + i * kPer + e;
                        L.cand_cnt[wbuf + off] = c[e];
                    }
                    wn += (uint32_t)__popcll(msk);
                }
            }
            }
            if (wn >= 64u) score_buffer(true);
        }
        if (t < t_last) __syncthreads();               // counters clear before tile t + 1 is consumed
    }

    score_buffer(false);                                // what is left of the item's candidates
    // top-k of the item: the wavefronts' lists (in LDS), merged by one thread
    const unsigned long long sc = block_sum<unsigned long long, NT>(scored, sh.red);   // has barriers
    if (tid == 0) {
        uint32_t* head = sh.head;
        for (int v = 0; v < (int)(NT / 64); ++v) head[v] = 0;
        for (uint32_t j = 0; j < kk; ++j) {
            int best = 0;
            for (int v = 1; v < (int)(NT / 64); ++v)
                if (better_hit(sh.wh[v][head[v]], sh.wid[v][head[v]], sh.wh[best][head[best]], sh.wid[best][head[best]]))
                    best = v;
            const uint32_t hh = head[best]++;
            const C c = (C)sh.wc[best][hh];
            const uint32_t id = sh.wid[best][hh];
            ps_hit o;
            o.id = id;
            o.n_b = (uint16_t)(id == 0xFFFFFFFFu ? 0 : Cnt<C>::nb(c));
            o.n_y = (uint16_t)(id == 0xFFFFFFFFu ? 0 : Cnt<C>::ny(c));
            o.sum_q = id == 0xFFFFFFFFu ? 0 : Cnt<C>::s(c);
            o.pad = 0;
            o.hyperscore = sh.wh[best][hh];
            out[j] = o;
        }
        if (sc) atomicAdd(&A.w.n_scored[s], sc);
    }
    for (uint32_t i = tid; i < (uint32_t)kHistBins; i += NT) {
        const int32_t v = L.hist[i];
        if (v) atomicAdd(&A.w.hist[(uint64_t)s * kHistBins + i], v);
    }
    if (tid == 0) {
        if (sh.acc_post) atomicAdd(&A.w.counters[kCtrPostings], sh.acc_post);
        if (sh.acc_look) atomicAdd(&A.w.counters[kCtrLookups], sh.acc_look);
        if (sh.acc_dpost) atomicAdd(&A.w.counters[kCtrDensePost], sh.acc_dpost);
        if (sh.acc_dreads) atomicAdd(&A.w.counters[kCtrDenseIds], sh.acc_dreads);
    }
    __syncthreads();
}

// Plain schedule: workgroup s searches spectrum s's whole window.  With one
// probe slot per thread the kernel asks for six resident wavefronts per SIMD
// (at most 80 VGPRs).
template <typename C, bool DUMP, uint32_t U, uint32_t NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(U == 1 ? 6 : 1, 8))) void k_scan_plain(ScanArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ ScanShared<NT> sh;
    ScanLds<C, NT> L(lds, A.kp.tile, A.kp.seg_cap);
    const uint32_t s = blockIdx.x;
    if (s >= A.sp.hdr->n) return;
    const SpecInfo inf = A.w.info[s];
    const bool wide = (inf.flags & kFlagWide) != 0;
    const bool skip = (inf.flags & (kFlagInvalid | kFlagOverflow)) || inf.hi <= inf.lo;
    if (wide != (A.want_wide != 0)) return;            // the other launch handles it
    if (A.per_item && skip) return;                    // no work item: nothing to write
    ps_hit* out = A.w.partial + (uint64_t)(A.per_item ? A.w.spec_item0[s] : s) * A.kp.top_k;
    if (skip) {
        if (threadIdx.x < A.kp.top_k) {
            ps_hit o; o.id = 0xFFFFFFFFu; o.n_b = o.n_y = 0; o.sum_q = 0; o.pad = 0; o.hyperscore = -INFINITY;
            out[threadIdx.x] = o;
        }
        return;
    }
    scan_item<C, DUMP, U, NT>(A, sh, L, s, inf.lo, inf.hi, out);
}

// Register slots per thread for a workgroup of nt threads that may hold
// seg_cap probe slots.
static uint32_t slots_per_thread(uint32_t seg_cap, uint32_t nt) {
    const uint32_t u = (seg_cap + nt - 1) / nt;
    return u <= 1 ? 1u : u == 2 ? 2u : u == 3 ? 3u : u == 4 ? 4u : 8u;
}

template <typename C, bool DUMP, uint32_t U, uint32_t NT>
static hipError_t launch_scan_plain_u(ScanArgs a, uint64_t n, hipStream_t stream) {
    const size_t lds = scan_lds_bytes(a.kp, sizeof(C) == 8);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_scan_plain<C, DUMP, U, NT>), dim3((uint32_t)n), dim3(NT), lds, stream, a);
    return hipGetLastError();
}

template <typename C, bool DUMP, uint32_t NT>
static hipError_t launch_scan_plain_t(ScanArgs a, uint64_t n, hipStream_t stream) {
    switch (slots_per_thread(a.kp.seg_cap, NT)) {
        case 1: return launch_scan_plain_u<C, DUMP, 1, NT>(a, n, stream);
        case 2: return launch_scan_plain_u<C, DUMP, 2, NT>(a, n, stream);
        case 3: return launch_scan_plain_u<C, DUMP, 3, NT>(a, n, stream);
        case 4: return launch_scan_plain_u<C, DUMP, 4, NT>(a, n, stream);
        default:
            if constexpr (NT == 256) return launch_scan_plain_u<C, DUMP, 8, NT>(a, n, stream);
            else return hipErrorInvalidValue;   // 512 threads hold every probe slot in 4 per thread
    }
}

// 64-bit counters take twice the LDS per candidate: they run in workgroups of
// 256 threads, halving the tile (down to one directory block) until it fits.
static KParams wide_params(const DevIndex& ix, KParams kp) {
    kp.nt = 256;
    while (kp.tile > (1u << ix.dir_shift) && scan_lds_bytes(kp, true) > kMaxLds) {
        kp.tile /= 2;
        kp.tile_shift -= 1;
    }
    return kp;
}

hipError_t launch_scan_plain(const DevIndex& ix, const DevSpectra& sp, const KParams& kp, const Work& w,
                             bool dump, bool per_item, bool wide_only, hipStream_t stream) {
    if (sp.n == 0) return hipSuccess;
    ScanArgs a{ix, sp, kp, w, 1u, 0u, per_item ? 1u : 0u};
    hipError_t e = hipSuccess;
    // narrow counters for every spectrum that proved it can use them, then wide
    if (!wide_only) {
        a.want_wide = 0;
        if (kp.nt == 512)
            e = dump ? launch_scan_plain_t<uint32_t, true, 512>(a, sp.n, stream)
                     : launch_scan_plain_t<uint32_t, false, 512>(a, sp.n, stream);
        else
            e = dump ? launch_scan_plain_t<uint32_t, true, 256>(a, sp.n, stream)
                     : launch_scan_plain_t<uint32_t, false, 256>(a, sp.n, stream);
        if (e != hipSuccess) return e;
    }
    a.want_wide = 1;
    a.kp = wide_params(ix, kp);
    e = dump ? launch_scan_plain_t<unsigned long long, true, 256>(a, sp.n, stream)
             : launch_scan_plain_t<unsigned long long, false, 256>(a, sp.n, stream);
    return e;
}

// ---------------------------------------------------------------------------
// persistent schedule: a work list of (spectrum, tile range) items and one
// resident grid that pops items from a device queue
// ---------------------------------------------------------------------------

struct ListArgs {
    DevSpectra sp;
    KParams kp;
    Work w;
    uint32_t tiles_per_item;
};

// Items per spectrum: ceil(tiles / tiles_per_item) for narrow-counter spectra,
// one slot for a wide-counter spectrum (filled by the plain wide kernel), none
// for invalid, overflowing or empty-window spectra.  spec_item0 is their
// exclusive prefix sum; spec_item0[n] is the total.  One workgroup.
// Items are aligned to the global grid of `span` = tile * tiles_per_item ids,
// so interior items start on directory blocks when span is a multiple of them.
__device__ __forceinline__ uint32_t items_of(const SpecInfo& inf, uint32_t tile, uint32_t tpi) {
    if ((inf.flags & (kFlagInvalid | kFlagOverflow)) || inf.hi <= inf.lo) return 0u;
    if (inf.flags & kFlagWide) return 1u;
    const uint32_t span = tile * tpi;
    return (inf.hi - 1) / span - inf.lo / span + 1;
}

__global__ __launch_bounds__(kBlock) void k_worklist(ListArgs A) {
    __shared__ unsigned long long s_part[kBlock];
    const uint64_t n = A.sp.hdr->n;
    const uint32_t tid = threadIdx.x;
    const uint64_t a = n * tid / kBlock, b = n * (tid + 1) / kBlock;
    unsigned long long sum = 0;
    for (uint64_t s = a; s < b; ++s) sum += items_of(A.w.info[s], A.kp.tile, A.tiles_per_item);
    s_part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        unsigned long long run = 0;
        for (int i = 0; i < kBlock; ++i) { const unsigned long long t = s_part[i]; s_part[i] = run; run += t; }
        A.w.spec_item0[n] = (uint32_t)run;
        A.w.counters[kCtrItems] = run;
    }
    __syncthreads();
    unsigned long long run = s_part[tid];
    for (uint64_t s = a; s < b; ++s) {
        A.w.spec_item0[s] = (uint32_t)run;
        run += items_of(A.w.info[s], A.kp.tile, A.tiles_per_item);
    }
}

hipError_t launch_worklist(const DevSpectra& sp, const KParams& kp, const Work& w, uint32_t tiles_per_item,
                           hipStream_t stream) {
    ListArgs a{sp, kp, w, tiles_per_item};
    hipLaunchKernelGGL(k_worklist, dim3(1), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

// With one probe slot per thread, ask for six resident wavefronts per SIMD
// (at most 80 VGPRs): with the LDS of the resident workgroups this is the
// occupancy the work-queue scan runs best at.
template <typename C, uint32_t U, uint32_t NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(U == 1 ? 6 : 1, 8)))
void k_scan_persistent(ScanArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ ScanShared<NT> sh;
    __shared__ uint32_t s_item;
    ScanLds<C, NT> L(lds, A.kp.tile, A.kp.seg_cap);
    const uint32_t n = (uint32_t)A.sp.hdr->n;
    const uint32_t total = A.w.spec_item0[n];
    const uint32_t tpi = A.tiles_per_item;
    while (true) {
        if (threadIdx.x == 0) s_item = (uint32_t)atomicAdd(&A.w.counters[kCtrQueue], 1ull);
        __syncthreads();
        const uint32_t g = s_item;
        __syncthreads();
        if (g >= total) break;                         // queue drained: every workgroup exits
        // spectrum of item g: the last s with spec_item0[s] <= g
        uint32_t lo = 0, hi = n;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (A.w.spec_item0[mid] <= g) lo = mid; else hi = mid;
        }
        const uint32_t s = lo;
        const SpecInfo inf = A.w.info[s];
        if (inf.flags & kFlagWide) continue;           // its slot is filled by the wide kernel
        const uint32_t span = tpi * A.kp.tile;
        const uint32_t blk = inf.lo / span + (g - A.w.spec_item0[s]);
        const uint32_t ida = max(inf.lo, blk * span);
        const uint32_t idb = min(inf.hi, (blk + 1) * span);
        scan_item<C, false, U, NT>(A, sh, L, s, ida, idb, A.w.partial + (uint64_t)g * A.kp.top_k);
    }
}

template <typename C, uint32_t U, uint32_t NT>
static hipError_t launch_persistent_u(ScanArgs a, uint32_t grid, hipStream_t stream) {
    const size_t lds = scan_lds_bytes(a.kp, sizeof(C) == 8);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_scan_persistent<C, U, NT>), dim3(grid), dim3(NT), lds, stream, a);
    return hipGetLastError();
}

template <uint32_t NT>
static hipError_t launch_persistent_t(ScanArgs a, uint32_t grid, hipStream_t stream) {
    switch (slots_per_thread(a.kp.seg_cap, NT)) {
        case 1: return launch_persistent_u<uint32_t, 1, NT>(a, grid, stream);
        case 2: return launch_persistent_u<uint32_t, 2, NT>(a, grid, stream);
        case 3: return launch_persistent_u<uint32_t, 3, NT>(a, grid, stream);
        case 4: return launch_persistent_u<uint32_t, 4, NT>(a, grid, stream);
        default:
            if constexpr (NT == 256) return launch_persistent_u<uint32_t, 8, NT>(a, grid, stream);
            else return hipErrorInvalidValue;
    }
}

hipError_t launch_scan_persistent(const DevIndex& ix, const DevSpectra& sp, const KParams& kp, const Work& w,
                                  uint32_t grid, uint32_t tiles_per_item, hipStream_t stream) {
    if (sp.n == 0) return hipSuccess;
    ScanArgs a{ix, sp, kp, w, tiles_per_item, 0u, 1u};
    hipError_t e = kp.nt == 512 ? launch_persistent_t<512>(a, grid, stream) : launch_persistent_t<256>(a, grid, stream);
    if (e != hipSuccess) return e;
    // spectra that need 64-bit counters: one workgroup per spectrum, slot = its item
    return launch_scan_plain(ix, sp, kp, w, false, true, true, stream);
}

// Allow every scan kernel the whole LDS once, before any launch or capture.
hipError_t init_kernel_attributes() {
#define PS_NARROW_FNS(U, NT)                                                                           \
        (const void*)k_scan_plain<uint32_t, false, U, NT>, (const void*)k_scan_plain<uint32_t, true, U, NT>, \
        (const void*)k_scan_persistent<uint32_t, U, NT>
#define PS_WIDE_FNS(U)                                                                                 \
        (const void*)k_scan_plain<unsigned long long, false, U, 256>,                                  \
        (const void*)k_scan_plain<unsigned long long, true, U, 256>
    const void* fns[] = {PS_NARROW_FNS(1, 256), PS_NARROW_FNS(2, 256), PS_NARROW_FNS(3, 256), PS_NARROW_FNS(4, 256),
                         PS_NARROW_FNS(8, 256), PS_NARROW_FNS(1, 512), PS_NARROW_FNS(2, 512), PS_NARROW_FNS(3, 512),
                         PS_NARROW_FNS(4, 512), PS_WIDE_FNS(1), PS_WIDE_FNS(2), PS_WIDE_FNS(3), PS_WIDE_FNS(4),
                         PS_WIDE_FNS(8)};
#undef PS_NARROW_FNS
#undef PS_WIDE_FNS
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ps

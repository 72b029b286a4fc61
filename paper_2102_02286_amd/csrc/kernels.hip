// kernels.hip -- the search path on gfx950.
//
//   k_prep     spectrum pre-processing (top-B peaks, integer intensities, m/z to
//              uDa, fragment-charge expansion to bin entries) and the precursor
//              window (filter_1 of Supplementary Algorithm 3)
//   k_scan     per work item (spectrum, id range): fragment-bin lookups to
//              posting segments (filter_2), streaming of postings into LDS
//              shared-peak counters tile by tile, then per tile the candidate
//              filter (shared peaks >= k), hyperscore, per-thread top-k and the
//              LDS score histogram (Supplementary Algorithm 3's score/heap)
//   k_merge    merge of partial top-k lists, Savitzky-Golay smoothed survival
//              function, linear tail fit and expect value (Superstep 4;
//              Supplementary Algorithm 4)
//
// Integer work is exact: counters are packed integer fields, the histogram is
// integer, and hyperscores come from host-built fp64 tables, so results do not
// depend on atomic order.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// First index in [lo, hi) with a[i] >= v, found by one wavefront: each round
// the 64 lanes probe evenly spaced positions and a ballot narrows the range
// 64-fold, so a segment of n postings costs ~log64(n) dependent loads.
// Must be called by all 64 lanes with identical (lo, hi, v).
__device__ __forceinline__ uint32_t wave_lower_bound(const uint32_t* a, uint32_t lo, uint32_t hi, uint32_t v) {
    const uint32_t lane = threadIdx.x & 63u;
    while (hi - lo > 64u) {
        uint32_t stride = (hi - lo + 63u) >> 6;
        uint32_t p = lo + lane * stride;
        bool pred = (p < hi) && (a[p] < v);
        uint32_t c = (uint32_t)__popcll(__ballot(pred));
        if (c == 0) return lo;
        uint32_t nlo = lo + (c - 1u) * stride + 1u;
        uint32_t nhi = min(hi, lo + c * stride);
        lo = nlo;
        hi = nhi;
    }
    uint32_t p = lo + lane;
    bool pred = (p < hi) && (a[p] < v);
    return lo + (uint32_t)__popcll(__ballot(pred));
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
    // scratch: kBlock/64 slots
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < kBlock / 64; ++i) r += scratch[i];
        scratch[0] = r;
    }
    __syncthreads();
    r = scratch[0];
    __syncthreads();
    return r;
}

// Packed shared-peak counters.  Narrow: [n_b:8 | n_y:8 | S:16] in 32 bits;
// wide: [n_b:16 | n_y:16 | S:32] in 64 bits.  The prep kernel proves per
// spectrum that no field can overflow before choosing the narrow form.
template <typename C> struct Cnt;
template <> struct Cnt<uint32_t> {
    __device__ static uint32_t inc(uint32_t is_y, uint32_t q) { return (is_y ? (1u << 16) : (1u << 24)) + q; }
    __device__ static uint32_t nb(uint32_t c) { return c >> 24; }
    __device__ static uint32_t ny(uint32_t c) { return (c >> 16) & 0xFFu; }
    __device__ static uint32_t s(uint32_t c) { return c & 0xFFFFu; }
};
template <> struct Cnt<unsigned long long> {
    __device__ static unsigned long long inc(uint32_t is_y, uint32_t q) {
        return (is_y ? (1ull << 32) : (1ull << 48)) + (unsigned long long)q;
    }
    __device__ static uint32_t nb(unsigned long long c) { return (uint32_t)(c >> 48); }
    __device__ static uint32_t ny(unsigned long long c) { return (uint32_t)(c >> 32) & 0xFFFFu; }
    __device__ static uint32_t s(unsigned long long c) { return (uint32_t)c; }
};

// Top-k of one wavefront, distributed over its lanes: lane j < k holds the
// j-th best candidate by (hyperscore desc, id asc).  An insertion is a ballot
// for the first lane the newcomer beats and a one-lane shift below it, so the
// list costs each lane one entry of registers instead of k.
__device__ __forceinline__ bool better_hit(double ha, uint32_t ia, double hb, uint32_t ib) {
    return ha > hb || (ha == hb && ia < ib);
}

template <typename C>
struct WaveTopK {
    double h;
    uint32_t id;
    C c;
    __device__ void init() { h = -INFINITY; id = 0xFFFFFFFFu; c = 0; }
    // Insert a wave-uniform candidate; every lane of the wavefront calls this.
    __device__ void insert(double xh, uint32_t xid, C xc, uint32_t k) {
        const uint32_t lane = threadIdx.x & 63u;
        const unsigned long long m = __ballot(lane < k && better_hit(xh, xid, h, id));
        if (m == 0) return;
        const uint32_t p = (uint32_t)__ffsll((long long)m) - 1u;
        const double uh = __shfl_up(h, 1, 64);
        const uint32_t uid = __shfl_up(id, 1, 64);
        const C uc = __shfl_up(c, 1, 64);
        if (lane > p && lane < k) { h = uh; id = uid; c = uc; }
        if (lane == p) { h = xh; id = xid; c = xc; }
    }
    // Insert every flagged lane's candidate that beats the current k-th best.
    __device__ void insert_lanes(bool flag, double ch, uint32_t cid, C cc, uint32_t k) {
        const double kh = __shfl(h, (int)k - 1, 64);
        const uint32_t kid = __shfl(id, (int)k - 1, 64);
        unsigned long long m = __ballot(flag && better_hit(ch, cid, kh, kid));
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            insert(__shfl(ch, l, 64), __shfl(cid, l, 64), __shfl(cc, l, 64), k);
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

struct PrepArgs {
    DevIndex ix;
    DevSpectra sp;
    KParams kp;
    Work w;
};

__global__ __launch_bounds__(kBlock) void k_prep(PrepArgs A) {
    __shared__ float s_mz[PS_MAX_PEAKS_IN];
    __shared__ float s_in[PS_MAX_PEAKS_IN];
    __shared__ uint32_t s_ent[PS_MAX_TOP_PEAKS * (PS_MAX_CHARGE - 1)];
    __shared__ uint32_t s_flag, s_imax_bits, s_mult;
    __shared__ unsigned long long s_red[kBlock / 64];
    const uint32_t tid = threadIdx.x;
    const KParams& kp = A.kp;

    const uint64_t n_batch = A.sp.hdr->n, nnz_batch = A.sp.hdr->nnz;
    for (uint64_t s = blockIdx.x; s < n_batch; s += gridDim.x) {
        const uint64_t p0 = A.sp.peak_off[s], p1 = A.sp.peak_off[s + 1];
        const int z = A.sp.charge[s];
        const double prec = A.sp.prec[s];
        if (tid == 0) {
            uint32_t bad = 0;
            if (!(p1 >= p0) || p1 - p0 > PS_MAX_PEAKS_IN || p1 > nnz_batch) bad = 1;
            if (z < 1 || z > (int)kp.max_charge) bad = 1;
            if (!(prec > 0.0) || !(prec <= 1e6)) bad = 1;   // also rejects NaN
            s_flag = bad;
            s_imax_bits = 0;
            s_mult = 0;
        }
        __syncthreads();
        const uint32_t np = s_flag ? 0u : (uint32_t)(p1 - p0);
        for (uint32_t i = tid; i < np; i += kBlock) {
            float m = A.sp.mz[p0 + i], v = A.sp.inten[p0 + i];
            s_mz[i] = m;
            s_in[i] = v;
            if (!(m > 0.0f) || !(m <= 3.0e38f) || !(v >= 0.0f) || !(v <= 3.0e38f)) atomicOr(&s_flag, 1u);
            else atomicMax(&s_imax_bits, __float_as_uint(v));   // ordered like floats for v >= 0
        }
        __syncthreads();
        const bool bad = s_flag != 0;
        const float imax = __uint_as_float(s_imax_bits);
        const uint32_t cmax = z > 2 ? (uint32_t)(z - 1) : 1u;
        const uint32_t keep = min(np, kp.top_peaks);
        const uint32_t n_ent = bad ? 0u : keep * cmax;
        uint32_t* gent = A.w.entries + s * (uint64_t)kp.ent_stride;
        // top-B by (intensity desc, m/z asc, input order asc): rank = number of better peaks
        if (!bad) {
            for (uint32_t i = tid; i < np; i += kBlock) {
                const float mi = s_mz[i], vi = s_in[i];
                uint32_t rank = 0;
                for (uint32_t j = 0; j < np; ++j) {
                    const float mj = s_mz[j], vj = s_in[j];
                    rank += (vj > vi) || (vj == vi && (mj < mi || (mj == mi && j < i)));
                }
                if (rank >= keep) continue;
                // integer intensity q in [1, 100] relative to the most intense peak
                uint32_t q = 1;
                if (imax > 0.0f) {
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
            uint32_t m = 0;
            for (uint32_t j = 0; j < n_ent; ++j) {
                const uint32_t ej = s_ent[j];
                if (ej == kEntryInvalid) continue;
                const uint32_t bj = ej >> 8;
                m += (bj >= bi && bj - bi <= span);
            }
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
                const int64_t prec_uda = round_half_up_pos(prec * 1e6);
                const int64_t mq = (int64_t)z * (prec_uda - kProtonUda);
                if (mq < 0) {
                    inf.flags = kFlagInvalid;
                } else {
                    const int64_t dm = kp.window_is_ppm ? (mq * kp.window) / 1000000 : kp.window;
                    // filter_1: ids with |M - M_q| <= dM  ->  [lo, hi)
                    const int64_t lo_m = mq - dm, hi_m = mq + dm;
                    uint64_t a = 0, b = A.ix.n_pep;
                    while (a < b) { uint64_t mid = (a + b) >> 1; if (A.ix.mass[mid] < lo_m) a = mid + 1; else b = mid; }
                    inf.lo = (uint32_t)a;
                    b = A.ix.n_pep;
                    while (a < b) { uint64_t mid = (a + b) >> 1; if (A.ix.mass[mid] <= hi_m) a = mid + 1; else b = mid; }
                    inf.hi = (uint32_t)a;
                    // worst-case field values for any candidate of this spectrum
                    const uint64_t nvalid = tot & 0xFFFFFFFFull, sq = tot >> 32;
                    const uint64_t width = (uint64_t)(2 * kp.tol + 1) * (uint64_t)kBinWidth;
                    const uint64_t kpe = A.ix.min_residue > 0 ? (width - 1) / (uint64_t)A.ix.min_residue + 1 : (1ull << 20);
                    uint64_t nbmax = nvalid * kpe;
                    const uint64_t by_len = (uint64_t)(A.ix.max_len > 0 ? A.ix.max_len - 1 : 0) * (uint64_t)s_mult;
                    if (by_len < nbmax) nbmax = by_len;
                    uint64_t smax = sq * 2ull * kpe;
                    if (200ull * nbmax < smax) smax = 200ull * nbmax;
                    if (!(nbmax <= 255 && smax <= 65535)) {
                        inf.flags |= kFlagWide;
                        if (!(nbmax < kLfSize && smax < kLsSize)) inf.flags |= kFlagOverflow;
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

constexpr uint32_t kCoopCap = 32;     // cooperative (long) segments per work item
constexpr uint32_t kChunkTiles = 16;  // tiles per boundary chunk of the cooperative segments
constexpr uint32_t kSentinel = 0xFFFFFFFFu;
constexpr uint32_t kBmCap = 4;        // dense-bin bitmap hits per work item (more go the posting route)
constexpr uint32_t kCandCap = 512;    // scored candidates buffered per tile before scoring

struct ScanShared {
    uint32_t nseg, nlight, ncoop, nhh, ncand;
    unsigned long long red[kBlock / 64];
    double wh[kBlock / 64][PS_MAX_TOP_K];          // per-wavefront top-k lists
    uint32_t wid[kBlock / 64][PS_MAX_TOP_K];
    unsigned long long wc[kBlock / 64][PS_MAX_TOP_K];
};

// LDS layout (dynamic):
//   counters (also the top-k merge area) | seg_cur | seg_end | seg_next | bitmap-hit slot |
//   seg_q | light list | bitmap-hit q | coop list | coop tile boundaries | histogram
template <typename C>
struct ScanLds {
    C* cnt;
    uint32_t* seg_cur;
    uint32_t* seg_end;
    uint32_t* seg_next;   // posting value at seg_cur (kSentinel when exhausted)
    uint32_t* hh_slot;    // bitmap slot of each dense-bin hit
    uint16_t* seg_q;
    uint16_t* light;
    uint16_t* hh_q;
    uint16_t* coop;
    uint32_t* bnd;        // [kCoopCap][kChunkTiles + 1]
    uint32_t* bmw;        // [kBmCap][2][tile/32 + 2] bitmap words of the current tile
    C* cand_cnt;          // [kCandCap] counters of candidates that passed the filter
    uint16_t* cand_idx;   // [kCandCap] their positions in the tile
    int32_t* hist;
    __device__ ScanLds(uint8_t* base, uint32_t tile, uint32_t segcap, uint32_t bmcap) {
        size_t o = 0;
        cnt = (C*)(base + o);
        o += ((size_t)tile * sizeof(C) + 15) & ~(size_t)15;
        cand_cnt = (C*)(base + o); o += (size_t)kCandCap * sizeof(C);
        seg_cur = (uint32_t*)(base + o); o += (size_t)segcap * 4;
        seg_end = (uint32_t*)(base + o); o += (size_t)segcap * 4;
        seg_next = (uint32_t*)(base + o); o += (size_t)segcap * 4;
        hh_slot = (uint32_t*)(base + o); o += (size_t)kBmCap * 4;
        bnd = (uint32_t*)(base + o); o += (size_t)kCoopCap * (kChunkTiles + 1) * 4;
        bmw = (uint32_t*)(base + o); o += (size_t)bmcap * 2 * (tile / 32 + 2) * 4;
        hist = (int32_t*)(base + o); o += (size_t)kHistBins * 4;
        seg_q = (uint16_t*)(base + o); o += (size_t)segcap * 2;
        light = (uint16_t*)(base + o); o += (size_t)segcap * 2;
        hh_q = (uint16_t*)(base + o); o += (size_t)kBmCap * 2;
        coop = (uint16_t*)(base + o); o += (size_t)kCoopCap * 2;
        cand_idx = (uint16_t*)(base + o);
    }
};

size_t scan_lds_bytes(const KParams& kp, bool wide) {
    const size_t csz = wide ? 8 : 4;
    size_t o = ((size_t)kp.tile * csz + 15) & ~(size_t)15;
    o += (size_t)kCandCap * csz;
    o += (size_t)kp.seg_cap * 12 + (size_t)kBmCap * 4 + (size_t)kCoopCap * (kChunkTiles + 1) * 4;
    o += (size_t)(kp.use_bitmaps ? kBmCap : 0) * 2 * (kp.tile / 32 + 2) * 4 + (size_t)kHistBins * 4;
    o += (size_t)kp.seg_cap * 4 + (size_t)kBmCap * 2 + (size_t)kCoopCap * 2 + (size_t)kCandCap * 2;
    return (o + 15) & ~(size_t)15;
}

// Hyperscore of one candidate that passed the filter: log10(n_b! n_y! S) from
// the fp64 tables, plus its histogram bin (width 0.1, last bin open).
template <typename C, bool DUMP>
__device__ __forceinline__ double score_one(const ScanArgs& A, ScanLds<C>& L, uint32_t s, uint32_t id, C c,
                                            uint32_t& scored) {
    const uint32_t nb = Cnt<C>::nb(c), ny = Cnt<C>::ny(c), sq = Cnt<C>::s(c);
    const double h = (A.ix.lf[nb] + A.ix.lf[ny]) + A.ix.ls[sq];
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

// One work item: spectrum s, candidate ids [ida, idb).  Writes the item's top
// hits to `out` (top_k entries) and adds its histogram and counts to the
// spectrum's global accumulators.
template <typename C, bool DUMP>
__device__ void scan_item(const ScanArgs& A, ScanShared& sh, ScanLds<C>& L, uint32_t s, uint32_t ida,
                          uint32_t idb, ps_hit* out) {
    const uint32_t tid = threadIdx.x;
    const KParams& kp = A.kp;
    const DevIndex& ix = A.ix;
    const uint32_t n_ent = A.w.info[s].n_ent;
    const uint32_t* ent = A.w.entries + (uint64_t)s * kp.ent_stride;
    const int T = kp.tol;
    const uint32_t width = (uint32_t)(2 * T + 1);

    if (tid == 0) { sh.nseg = 0; sh.nlight = 0; sh.ncoop = 0; sh.nhh = 0; }
    for (uint32_t i = tid; i < (uint32_t)kHistBins; i += kBlock) L.hist[i] = 0;
    __syncthreads();

    // filter_2, part 1: every (entry, bin offset) -> posting run inside [ida, idb).
    // Dense bins become bitmap hits; long runs are streamed cooperatively; the
    // rest are walked by one thread each.
    unsigned long long lookups = 0, postings = 0;
    const uint32_t npairs = n_ent * width;
    for (uint32_t k = tid; k < npairs; k += kBlock) {
        const uint32_t e = ent[k / width];
        if (e == kEntryInvalid) continue;
        const int64_t bin = (int64_t)(e >> 8) + (int64_t)(k % width) - T;
        if (bin < 0 || bin >= (int64_t)ix.n_bins) continue;
        ++lookups;
        const uint32_t* d = ix.dir + (uint64_t)bin * (ix.dir_nblk + 1);
        // first posting with id >= ida / idb: exact when the id is block aligned,
        // else a search inside one block of the bin
        const uint32_t ka = ida >> ix.dir_shift, kb = idb >> ix.dir_shift;
        const uint32_t a0 = d[ka];
        const uint32_t s0 = (ida & ((1u << ix.dir_shift) - 1)) ? lower_bound_u32(ix.post, a0, d[ka + 1], ida << 1) : a0;
        const uint32_t b0 = d[kb];
        const uint32_t s1 = (idb & ((1u << ix.dir_shift) - 1)) ? lower_bound_u32(ix.post, b0, d[kb + 1], idb << 1) : b0;
        if (s1 <= s0) continue;
        postings += s1 - s0;
        const uint16_t q = (uint16_t)(e & 0xFFu);
        if (kp.use_bitmaps) {
            const int32_t hs = ix.heavy_slot[bin];
            if (hs >= 0) {
                const uint32_t h = atomicAdd(&sh.nhh, 1u);
                if (h < kBmCap) {
                    L.hh_slot[h] = (uint32_t)hs;
                    L.hh_q[h] = q;
                    continue;
                }
            }
        }
        const uint32_t slot = atomicAdd(&sh.nseg, 1u);
        L.seg_cur[slot] = s0;
        L.seg_end[slot] = s1;
        L.seg_q[slot] = q;
        if (s1 - s0 > kp.coop_min) {
            const uint32_t c = atomicAdd(&sh.ncoop, 1u);
            if (c < kCoopCap) { L.coop[c] = (uint16_t)slot; continue; }
        }
        L.seg_next[slot] = ix.post[s0];
        L.light[atomicAdd(&sh.nlight, 1u)] = (uint16_t)slot;
    }
    __syncthreads();
    const uint32_t nlight = sh.nlight, nhh = min(sh.nhh, kBmCap);
    const uint32_t ncoop = min(sh.ncoop, kCoopCap);
    // no posting in range: every counter stays 0 < k_min, nothing can be scored
    const uint32_t id_end = (nlight + ncoop + nhh) ? idb : ida;

    WaveTopK<C> top;
    top.init();
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t kk = kp.top_k;
    uint32_t scored = 0;
    const uint32_t kmin = kp.min_shared;
    const uint64_t bmw = ix.bm_words;
    (void)bmw;
    if (id_end > ida)
        for (uint32_t i = tid; i < kp.tile; i += kBlock) L.cnt[i] = 0;
    if (tid == 0) sh.ncand = 0;
    const uint32_t wpt = kp.tile / 32 + 2;
    __syncthreads();
    for (uint32_t tc0 = ida; tc0 < id_end; tc0 += kChunkTiles * kp.tile) {
        const uint32_t left = id_end - tc0;
        const uint32_t nch = min(kChunkTiles, (left + kp.tile - 1) / kp.tile);
        // tile boundaries of every cooperative run in this chunk
        for (uint32_t q = tid; q < ncoop * nch; q += kBlock) {
            const uint32_t c = q / nch, k = q - c * nch;
            const uint32_t sg = L.coop[c];
            const uint32_t lim = min(id_end, tc0 + (k + 1) * kp.tile) << 1;
            L.bnd[c * (kChunkTiles + 1) + k + 1] = lower_bound_u32(ix.post, L.seg_cur[sg], L.seg_end[sg], lim);
        }
        for (uint32_t c = tid; c < ncoop; c += kBlock) L.bnd[c * (kChunkTiles + 1)] = L.seg_cur[L.coop[c]];
        __syncthreads();
        for (uint32_t k = 0; k < nch; ++k) {
            const uint32_t tb = tc0 + k * kp.tile;
            const uint32_t te = min(id_end, tb + kp.tile);
            const uint32_t nt = te - tb;
            const uint32_t lim = te << 1;
            if (tid == 0) sh.ncand = 0;
            // this tile's words of the dense-bin bitmaps, staged in LDS
            for (uint32_t q = tid; q < nhh * 2 * wpt; q += kBlock) {
                const uint32_t h = q / (2 * wpt), r = q - h * 2 * wpt;
                const uint32_t half = r / wpt, wi = r - half * wpt;
                const uint64_t word = (uint64_t)(tb >> 5) + wi;
                L.bmw[q] = word < bmw ? ix.bitmaps[(uint64_t)L.hh_slot[h] * 2 * bmw + half * bmw + word] : 0u;
            }
            // short runs: one thread each; the next posting id is cached in LDS so a
            // run with nothing in this tile costs no global load
            for (uint32_t j = tid; j < nlight; j += kBlock) {
                const uint32_t sg = L.light[j];
                uint32_t nx = L.seg_next[sg];
                if (nx >= lim) continue;
                uint32_t cur = L.seg_cur[sg];
                const uint32_t end = L.seg_end[sg];
                const uint32_t q = L.seg_q[sg];
                atomicAdd(&L.cnt[(nx >> 1) - tb], Cnt<C>::inc(nx & 1u, q));
                ++cur;
                while (true) {
                    if (cur >= end) { nx = kSentinel; break; }
                    const uint32_t p0 = ix.post[cur];
                    const uint32_t p1 = cur + 1 < end ? ix.post[cur + 1] : kSentinel;
                    const uint32_t p2 = cur + 2 < end ? ix.post[cur + 2] : kSentinel;
                    const uint32_t p3 = cur + 3 < end ? ix.post[cur + 3] : kSentinel;
                    if (p0 >= lim) { nx = p0; break; }
                    atomicAdd(&L.cnt[(p0 >> 1) - tb], Cnt<C>::inc(p0 & 1u, q));
                    ++cur;
                    if (p1 >= lim) { nx = p1; break; }
                    atomicAdd(&L.cnt[(p1 >> 1) - tb], Cnt<C>::inc(p1 & 1u, q));
                    ++cur;
                    if (p2 >= lim) { nx = p2; break; }
                    atomicAdd(&L.cnt[(p2 >> 1) - tb], Cnt<C>::inc(p2 & 1u, q));
                    ++cur;
                    if (p3 >= lim) { nx = p3; break; }
                    atomicAdd(&L.cnt[(p3 >> 1) - tb], Cnt<C>::inc(p3 & 1u, q));
                    ++cur;
                }
                L.seg_cur[sg] = cur;
                L.seg_next[sg] = nx;
            }
            // long runs: the whole workgroup streams this tile's part, coalesced
            for (uint32_t c = 0; c < ncoop; ++c) {
                const uint32_t b0 = L.bnd[c * (kChunkTiles + 1) + k], b1 = L.bnd[c * (kChunkTiles + 1) + k + 1];
                const uint32_t q = L.seg_q[L.coop[c]];
                uint32_t i = b0 + tid;
                for (; i + 3 * kBlock < b1; i += 4 * kBlock) {
                    const uint32_t p0 = ix.post[i], p1 = ix.post[i + kBlock];
                    const uint32_t p2 = ix.post[i + 2 * kBlock], p3 = ix.post[i + 3 * kBlock];
                    atomicAdd(&L.cnt[(p0 >> 1) - tb], Cnt<C>::inc(p0 & 1u, q));
                    atomicAdd(&L.cnt[(p1 >> 1) - tb], Cnt<C>::inc(p1 & 1u, q));
                    atomicAdd(&L.cnt[(p2 >> 1) - tb], Cnt<C>::inc(p2 & 1u, q));
                    atomicAdd(&L.cnt[(p3 >> 1) - tb], Cnt<C>::inc(p3 & 1u, q));
                }
                for (; i < b1; i += kBlock) {
                    const uint32_t p = ix.post[i];
                    atomicAdd(&L.cnt[(p >> 1) - tb], Cnt<C>::inc(p & 1u, q));
                }
            }
            __syncthreads();
            // candidate filter: counters (plus dense bins from the staged bitmap
            // words) are read and cleared for the next tile; candidates with at
            // least k_min shared peaks are buffered for scoring
            const uint32_t w0 = tb >> 5;
            for (uint32_t base = wave * 64u; base < nt; base += kBlock) {   // wave-uniform trip count
                const uint32_t i = base + lane;
                bool ovf = false;
                C c = 0;
                if (i < nt) {
                    c = L.cnt[i];
                    L.cnt[i] = 0;
                    const uint32_t id = tb + i;
                    for (uint32_t h = 0; h < nhh; ++h) {
                        const uint32_t* bw = L.bmw + h * 2 * wpt;
                        const uint32_t wd = (id >> 5) - w0, sh5 = id & 31u;
                        const uint32_t q = L.hh_q[h];
                        if ((bw[wd] >> sh5) & 1u) c += Cnt<C>::inc(0u, q);
                        if ((bw[wpt + wd] >> sh5) & 1u) c += Cnt<C>::inc(1u, q);
                    }
                    if (Cnt<C>::nb(c) + Cnt<C>::ny(c) >= kmin) {
                        const uint32_t slot = atomicAdd(&sh.ncand, 1u);
                        if (slot < kCandCap) {
                            L.cand_idx[slot] = (uint16_t)i;
                            L.cand_cnt[slot] = c;
                        } else {
                            ovf = true;                 // buffer full: score in place below
                        }
                    }
                }
                if (__ballot(ovf)) {
                    const double h = ovf ? score_one<C, DUMP>(A, L, s, tb + i, c, scored) : -INFINITY;
                    top.insert_lanes(ovf, h, tb + i, c, kk);
                }
            }
            __syncthreads();
            // hyperscore, histogram, top-k over the buffered candidates
            const uint32_t ncand = min(sh.ncand, kCandCap);
            for (uint32_t base = wave * 64u; base < ncand; base += kBlock) {
                const uint32_t j = base + lane;
                const bool ok = j < ncand;
                const C c = ok ? L.cand_cnt[j] : (C)0;
                const uint32_t id = ok ? tb + L.cand_idx[j] : 0u;
                const double h = ok ? score_one<C, DUMP>(A, L, s, id, c, scored) : -INFINITY;
                top.insert_lanes(ok, h, id, c, kk);
            }
            __syncthreads();
        }
        for (uint32_t c = tid; c < ncoop; c += kBlock) L.seg_cur[L.coop[c]] = L.bnd[c * (kChunkTiles + 1) + nch];
        __syncthreads();
    }

    // top-k of the item: the wavefronts' lists, merged by one thread
    if (lane < kk) {
        sh.wh[wave][lane] = top.h;
        sh.wid[wave][lane] = top.id;
        sh.wc[wave][lane] = (unsigned long long)top.c;
    }
    const unsigned long long sc = block_sum<unsigned long long>(scored, sh.red);   // has barriers
    if (tid == 0) {
        uint32_t head[kBlock / 64];
        for (int v = 0; v < kBlock / 64; ++v) head[v] = 0;
        for (uint32_t j = 0; j < kk; ++j) {
            int best = 0;
            for (int v = 1; v < kBlock / 64; ++v)
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
    for (uint32_t i = tid; i < (uint32_t)kHistBins; i += kBlock) {
        const int32_t v = L.hist[i];
        if (v) atomicAdd(&A.w.hist[(uint64_t)s * kHistBins + i], v);
    }
    const unsigned long long pl = block_sum<unsigned long long>(postings, sh.red);
    const unsigned long long lk = block_sum<unsigned long long>(lookups, sh.red);
    if (tid == 0) {
        if (pl) atomicAdd(&A.w.counters[kCtrPostings], pl);
        if (lk) atomicAdd(&A.w.counters[kCtrLookups], lk);
    }
    __syncthreads();
}

// Plain schedule: workgroup s searches spectrum s's whole window.
template <typename C, bool DUMP>
__global__ __launch_bounds__(kBlock) void k_scan_plain(ScanArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ ScanShared sh;
    ScanLds<C> L(lds, A.kp.tile, A.kp.seg_cap, A.kp.use_bitmaps ? kBmCap : 0);
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
    scan_item<C, DUMP>(A, sh, L, s, inf.lo, inf.hi, out);
}

template <typename C, bool DUMP>
static hipError_t launch_scan_plain_t(ScanArgs a, uint64_t n, hipStream_t stream) {
    const size_t lds = scan_lds_bytes(a.kp, sizeof(C) == 8);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_scan_plain<C, DUMP>), dim3((uint32_t)n), dim3(kBlock), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_scan_plain(const DevIndex& ix, const DevSpectra& sp, const KParams& kp, const Work& w,
                             bool dump, bool per_item, bool wide_only, hipStream_t stream) {
    if (sp.n == 0) return hipSuccess;
    ScanArgs a{ix, sp, kp, w, 1u, 0u, per_item ? 1u : 0u};
    hipError_t e = hipSuccess;
    // narrow counters for every spectrum that proved it can use them, then wide
    if (!wide_only) {
        a.want_wide = 0;
        e = dump ? launch_scan_plain_t<uint32_t, true>(a, sp.n, stream) : launch_scan_plain_t<uint32_t, false>(a, sp.n, stream);
        if (e != hipSuccess) return e;
    }
    a.want_wide = 1;
    // 64-bit counters take twice the LDS per candidate: halve the tile until it fits
    while (a.kp.tile > 1024 && scan_lds_bytes(a.kp, true) > kMaxLds) a.kp.tile /= 2;
    e = dump ? launch_scan_plain_t<unsigned long long, true>(a, sp.n, stream)
             : launch_scan_plain_t<unsigned long long, false>(a, sp.n, stream);
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

template <typename C>
__global__ __launch_bounds__(kBlock) void k_scan_persistent(ScanArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ ScanShared sh;
    __shared__ uint32_t s_item;
    ScanLds<C> L(lds, A.kp.tile, A.kp.seg_cap, A.kp.use_bitmaps ? kBmCap : 0);
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
        scan_item<C, false>(A, sh, L, s, ida, idb, A.w.partial + (uint64_t)g * A.kp.top_k);
    }
}

template <typename C>
static hipError_t launch_persistent_t(ScanArgs a, uint32_t grid, hipStream_t stream) {
    const size_t lds = scan_lds_bytes(a.kp, sizeof(C) == 8);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_scan_persistent<C>), dim3(grid), dim3(kBlock), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_scan_persistent(const DevIndex& ix, const DevSpectra& sp, const KParams& kp, const Work& w,
                                  uint32_t grid, uint32_t tiles_per_item, hipStream_t stream) {
    if (sp.n == 0) return hipSuccess;
    ScanArgs a{ix, sp, kp, w, tiles_per_item, 0u, 1u};
    hipError_t e = launch_persistent_t<uint32_t>(a, grid, stream);
    if (e != hipSuccess) return e;
    // spectra that need 64-bit counters: one workgroup per spectrum, slot = its item
    return launch_scan_plain(ix, sp, kp, w, false, true, true, stream);
}

// ---------------------------------------------------------------------------
// merge: partial top-k -> hits; histogram -> smoothed survival -> tail fit -> e-value
// ---------------------------------------------------------------------------

struct MergeArgs {
    DevIndex ix;
    DevSpectra sp;
    KParams kp;
    Work w;
    uint32_t per_item;   // 1: partial lists per work item (spec_item0 ranges); 0: one per spectrum
};

__global__ __launch_bounds__(kBlock) void k_merge(MergeArgs A) {
    __shared__ long long s_num[kHistBins];
    __shared__ long long s_tail[kHistBins];
    __shared__ long long s_redl[kBlock / 64];
    __shared__ ps_hit s_top[PS_MAX_TOP_K];
    __shared__ int s_mode;
    __shared__ unsigned long long s_modekey;
    const uint32_t tid = threadIdx.x;
    const uint32_t K = A.kp.top_k;
    const uint64_t n_batch = A.sp.hdr->n;
    for (uint64_t s = blockIdx.x; s < n_batch; s += gridDim.x) {
        const SpecInfo inf = A.w.info[s];
        const bool invalid = (inf.flags & kFlagInvalid) != 0;
        const bool overflow = (inf.flags & kFlagOverflow) != 0;
        // ---- top-k merge (thread 0, insertion; lists are short)
        if (tid == 0) {
            for (uint32_t j = 0; j < K; ++j) {
                s_top[j].id = 0xFFFFFFFFu; s_top[j].n_b = s_top[j].n_y = 0; s_top[j].sum_q = 0;
                s_top[j].pad = 0; s_top[j].hyperscore = -INFINITY;
            }
            uint64_t i0 = s, i1 = s + 1;
            if (A.per_item) { i0 = A.w.spec_item0[s]; i1 = A.w.spec_item0[s + 1]; }
            if (!invalid && !overflow) {
                for (uint64_t it = i0; it < i1; ++it) {
                    const ps_hit* src = A.w.partial + it * K;
                    for (uint32_t j = 0; j < K; ++j) {
                        ps_hit c = src[j];
                        if (c.id == 0xFFFFFFFFu) break;
                        // insert into s_top (sorted by hyperscore desc, id asc)
                        if (!(c.hyperscore > s_top[K - 1].hyperscore ||
                              (c.hyperscore == s_top[K - 1].hyperscore && c.id < s_top[K - 1].id)))
                            continue;
                        int p = (int)K - 1;
                        while (p > 0 && (c.hyperscore > s_top[p - 1].hyperscore ||
                                         (c.hyperscore == s_top[p - 1].hyperscore && c.id < s_top[p - 1].id))) {
                            s_top[p] = s_top[p - 1];
                            --p;
                        }
                        s_top[p] = c;
                    }
                }
            }
        }
        __syncthreads();
        const unsigned long long N = (invalid || overflow) ? 0ull : A.w.n_scored[s];
        const double h1 = s_top[0].hyperscore;
        // ---- Savitzky-Golay (-3, 12, 17, 12, -3)/35 numerators, exact in integers
        const int32_t* hg = A.w.hist + s * (uint64_t)kHistBins;
        long long part = 0;
        for (int j = tid; j < kHistBins; j += kBlock) {
            long long acc = 0;
            const int c[5] = {-3, 12, 17, 12, -3};
            for (int t = -2; t <= 2; ++t) {
                int i = j + t;
                if (i >= 0 && i < kHistBins && N) acc += (long long)c[t + 2] * (long long)hg[i];
            }
            if (acc < 0) acc = 0;
            s_num[j] = acc;
            part += acc;
        }
        // total
        for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o, 64);
        if ((tid & 63) == 0) s_redl[tid >> 6] = part;
        if (tid == 0) s_modekey = 0;
        __syncthreads();
        long long total = 0;
        for (int i = 0; i < kBlock / 64; ++i) total += s_redl[i];
        // mode: largest numerator, lowest index on ties -> max of (value << 9 | (511 - j))
        for (int j = tid; j < kHistBins; j += kBlock)
            atomicMax(&s_modekey, ((unsigned long long)s_num[j] << 9) | (unsigned long long)(kHistBins - 1 - j));
        __syncthreads();
        if (tid == 0) {
            s_mode = kHistBins - 1 - (int)(s_modekey & 511ull);
            long long run = 0;
            for (int j = kHistBins - 1; j >= 0; --j) { run += s_num[j]; s_tail[j] = run; }
        }
        __syncthreads();
        int status = PS_STATUS_OK;
        double ev = __builtin_nan("");
        if (invalid) status = PS_STATUS_INVALID;
        else if (overflow) status = PS_STATUS_OVERFLOW;
        else if (N == 0) status = PS_STATUS_NO_HITS;
        // ---- least-squares fit of log10 survival over [mode, bin(H1) - 1]
        double sx = 0, sy = 0, sxx = 0, sxy = 0, cnt = 0;
        if (status == PS_STATUS_OK && total > 0) {
            const double hb = floor(10.0 * h1);
            const int jh = hb >= (double)(kHistBins - 1) ? kHistBins - 1 : (int)hb;
            for (int j = s_mode + (int)tid; j <= jh - 1; j += kBlock) {
                const long long t = s_tail[j];
                if (t <= 0) continue;
                const double x = 0.1 * (double)j;
                const double y = log10((double)t / (double)total);
                sx += x; sy += y; sxx += x * x; sxy += x * y; cnt += 1.0;
            }
        }
        double v[5] = {sx, sy, sxx, sxy, cnt};
        __shared__ double s_v[5][kBlock / 64];
        for (int k = 0; k < 5; ++k) {
            double x = v[k];
            for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
            if ((tid & 63) == 0) s_v[k][tid >> 6] = x;
        }
        __syncthreads();
        if (tid == 0) {
            double t[5];
            for (int k = 0; k < 5; ++k) { t[k] = 0; for (int i = 0; i < kBlock / 64; ++i) t[k] += s_v[k][i]; }
            if (status == PS_STATUS_OK) {
                const double n = t[4];
                if (n < 3.0) {
                    status = PS_STATUS_FEW_POINTS;
                } else {
                    const double num = n * t[3] - t[0] * t[1];
                    const double den = n * t[2] - t[0] * t[0];
                    const double w = num / den;
                    const double b = (t[1] - w * t[0]) / n;
                    if (!(w < 0.0)) status = PS_STATUS_BAD_SLOPE;
                    else ev = (double)N * pow(10.0, w * h1 + b);
                }
            }
            ps_stat st;
            st.n_window = (invalid) ? 0ull : (unsigned long long)(inf.hi - inf.lo);
            st.n_scored = N;
            st.evalue = ev;
            st.status = status;
            st.pad = 0;
            A.w.stats[s] = st;
        }
        for (uint32_t j = tid; j < K; j += kBlock) A.w.hits[s * K + j] = s_top[j];
        __syncthreads();
    }
}

hipError_t launch_merge(const DevIndex& ix, const DevSpectra& sp, const KParams& kp, const Work& w,
                        bool per_item, hipStream_t stream) {
    if (sp.n == 0) return hipSuccess;
    MergeArgs a{ix, sp, kp, w, per_item ? 1u : 0u};
    uint64_t grid = sp.n < (1u << 20) ? sp.n : (1u << 20);
    hipLaunchKernelGGL(k_merge, dim3((uint32_t)grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

// Allow every scan kernel the whole LDS once, before any launch or capture.
hipError_t init_kernel_attributes() {
    const void* fns[] = {
        (const void*)k_scan_plain<uint32_t, false>, (const void*)k_scan_plain<uint32_t, true>,
        (const void*)k_scan_plain<unsigned long long, false>, (const void*)k_scan_plain<unsigned long long, true>,
        (const void*)k_scan_persistent<uint32_t>,
    };
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ps

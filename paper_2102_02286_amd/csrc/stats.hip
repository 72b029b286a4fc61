// stats.hip -- the per-spectrum statistics after the posting scan, on gfx950.
//
//   k_merge    top-k of a spectrum's partial lists (one per work item), then
//              the Savitzky-Golay smoothed survival function of its score
//              histogram, the linear tail fit (or the log-Weibull fit) and the
//              expect value (Superstep 4; Supplementary Algorithm 4)
//   k_assemble the same statistics over the results of G database partitions:
//              histogram addition (and the shift of sampled records) and a
//              G-way top-k merge first (Superstep 4)
//   k_sample   the 256-byte sampled record of a histogram (Sampling section)
//
// Each spectrum is handled by one wavefront, four per workgroup, with no block
// barriers and no LDS: lane l holds histogram bins 8 l .. 8 l + 7, neighbours
// and suffix sums cross lanes by shuffles, and the top k of sorted lists is a
// k-round tournament of wave-wide maxima.  k_merge and k_assemble share the
// expect-value code, so an assembled result equals the whole-database search
// bit for bit.
#include <hip/hip_runtime.h>

#include <cstring>

#include "internal.h"

namespace ps {

namespace {

constexpr uint32_t kStatWaves = kBlock / 64;   // spectra per workgroup

__device__ __forceinline__ void empty_hit(ps_hit& h) {
    h.id = 0xFFFFFFFFu; h.n_b = h.n_y = 0; h.sum_q = 0; h.pad = 0; h.hyperscore = -INFINITY;
}

__device__ __forceinline__ long long wave_sum_i64(long long x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ uint32_t wave_or_u32(uint32_t x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x |= (uint32_t)__shfl_xor((int)x, o, 64);
    return x;
}

// Sum of a double over the wavefront in one fixed order (a tree to lane 0),
// then broadcast, so every lane holds the same bits.
__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_down(x, o, 64);
    return __shfl(x, 0, 64);
}

// Wave-wide maximum of a 64-bit key.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

// Order of hits as one 128-bit key (hi, lo), larger first: hyperscore
// descending, then id ascending.  Hyperscores are >= 0 or -inf (empty), so the
// bits of a finite one plus 1 order like the values and -inf becomes 0; lo is
// the complemented id, so an empty hit (id UINT32_MAX) is (0, 0), the smallest.
struct HitKey {
    unsigned long long hi;
    uint32_t lo;
    uint32_t src;      // where the hit came from (list * k + position)
};

__device__ __forceinline__ HitKey hit_key(double h, uint32_t id, uint32_t src) {
    HitKey k;
    k.hi = h == -INFINITY ? 0ull : (unsigned long long)__double_as_longlong(h) + 1ull;
    k.lo = 0xFFFFFFFFu - id;
    k.src = src;
    return k;
}

__device__ __forceinline__ bool key_greater(const HitKey& a, const HitKey& b) {
    return a.hi > b.hi || (a.hi == b.hi && a.lo > b.lo);
}

// The largest key of the wavefront, in every lane (keys of distinct hits differ).
__device__ __forceinline__ HitKey wave_best(HitKey k) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        HitKey w;
        w.hi = __shfl_xor(k.hi, o, 64);
        w.lo = (uint32_t)__shfl_xor((int)k.lo, o, 64);
        w.src = (uint32_t)__shfl_xor((int)k.src, o, 64);
        if (key_greater(w, k)) k = w;
    }
    return k;
}

// Top k of L lists of k hits each, every list sorted by (hyperscore desc, id
// asc) with empty hits last.  key(c) is the hit at list c / k, position c % k
// (with its id as the merged result reports it).  Round r finds the best hit
// not yet taken; lane r keeps it.  With at most 64 lists lane a walks list a
// with a cursor; with more, every lane looks, in each of its lists, for the
// first hit worse than the last winner (ids are distinct, so the order is
// total).  Returns in lane r < k the source index of the r-th hit, or
// UINT32_MAX where fewer than r + 1 hits exist.
template <typename Key>
__device__ uint32_t wave_top_k(uint32_t L, uint32_t k, Key key) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t mine = 0xFFFFFFFFu;
    if (L <= 64) {
        uint32_t cur = 0;
        for (uint32_t r = 0; r < k; ++r) {
            HitKey c{0ull, 0u, 0xFFFFFFFFu};
            if (lane < L && cur < k) c = key(lane * k + cur);
            const HitKey w = wave_best(c);
            if (w.hi == 0 && w.lo == 0) break;          // only empty hits remain (wave-uniform)
            if (w.src == lane * k + cur) ++cur;
            if (lane == r) mine = w.src;
        }
        return mine;
    }
    HitKey prev{~0ull, 0xFFFFFFFFu, 0xFFFFFFFFu};     // above every hit
    for (uint32_t r = 0; r < k; ++r) {
        HitKey best{0ull, 0u, 0xFFFFFFFFu};
        for (uint32_t a = lane; a < L; a += 64) {
            // the list is sorted: keys better than prev form a prefix; find its end,
            // then step over prev itself if it came from this list
            uint32_t lo = 0, hi = k;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (key_greater(key(a * k + mid), prev)) lo = mid + 1; else hi = mid;
            }
            uint32_t p = lo;
            if (p < k && !key_greater(prev, key(a * k + p))) ++p;   // equal to prev: taken already
            if (p < k) {
                const HitKey c = key(a * k + p);
                if (key_greater(c, best)) best = c;
            }
        }
        const HitKey w = wave_best(best);
        if (w.hi == 0 && w.lo == 0) break;
        prev = w;
        if (lane == r) mine = w.src;
    }
    return mine;
}

// First bin of the window of PS_SAMPLE_BINS bins the Sampling section keeps
// (ps_sample), for a histogram held as bins 8 lane .. 8 lane + 7 in v[] (all
// counts >= 0): the floored mean of the three largest counts' bins (ties: the
// lower bin), the window reaching down to the first nonzero bin but no further
// than PS_SAMPLE_HEAD bins below that mean, and ending at bin 511 at the
// latest.  -1 when every count is 0.  Every lane calls it; the result is the
// same in every lane.
__device__ int sample_window_lo(const int32_t v[8]) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t used = 0, sum = 0, t = 0;
    for (int r = 0; r < 3; ++r) {
        unsigned long long best = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const unsigned long long key =
                ((unsigned long long)(uint32_t)v[i] << 32) | (uint32_t)(kHistBins - 1 - (8u * lane + i));
            if (v[i] > 0 && !((used >> i) & 1u) && key > best) best = key;
        }
        best = wave_max_u64(best);
        if (best == 0) break;                                   // wave-uniform
        const uint32_t bin = (uint32_t)(kHistBins - 1) - (uint32_t)(best & 0xFFFFFFFFull);
        if (bin / 8u == lane) used |= 1u << (bin % 8u);
        sum += bin;
        ++t;
    }
    if (t == 0) return -1;
    uint32_t first = kHistBins;
#pragma unroll
    for (int i = 7; i >= 0; --i)
        if (v[i] > 0) first = 8u * lane + i;
    first = wave_min_u32(first);
    const int mean = (int)(sum / t);
    const int lo = (int)first > mean - PS_SAMPLE_HEAD ? (int)first : mean - PS_SAMPLE_HEAD;
    return min(lo, kHistBins - PS_SAMPLE_BINS);
}

// The window the log-Weibull fit uses for the histogram in h[] (negative
// counts, which a search never writes, count as empty); -1 unless FIT is
// the log-Weibull one.
template <int FIT>
__device__ __forceinline__ int fit_window(const int32_t h[8]) {
    if constexpr (FIT != PS_FIT_GUMBEL) return -1;
    int32_t v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = h[i] > 0 ? h[i] : 0;
    return sample_window_lo(v);
}

// Fit of one spectrum's expect-value model (Superstep 4) to its histogram,
// bins 8 lane .. 8 lane + 7 in h[]: Savitzky-Golay smoothing with
// (-3, 12, 17, 12, -3)/35 (the integer numerators are kept, negatives set to 0;
// the factor 1/35 cancels), the survival function, then either the
// least-squares line w x + b of its log10 from the smoothed mode (lowest bin on
// ties) to the bin below the top hit, giving arg = w h1 + b for
// ev = N * 10^arg, or the log-Weibull (Gumbel) location and scale from the
// moments of the smoothed histogram restricted to the window a sampled record
// keeps (Sampling section; its first bin win_lo, from sample_window_lo on the
// same histogram, -1 if empty; bin centres 0.1 j + 0.05), giving
// arg = (h1 - mu) / beta for ev = N * (1 - exp(-exp(-arg))).  The exponential
// itself is taken by k_finish_evalue, one thread per spectrum, so that its
// registers are not held by every lane here.  `status` enters as OK, INVALID,
// OVERFLOW or NO_HITS; only OK is refined (to FEW_POINTS or BAD_SLOPE), and arg
// is NaN unless the status stays OK.  Every lane of the wavefront calls it; the
// results are the same in every lane.  `tl` is this wavefront's LDS area of
// 8 x 64 survival sums (bin 8 l + i at tl[64 i + l]), from which the fit range
// is dealt out to consecutive lanes.
template <int FIT>
__device__ void fit_wave(const int32_t h[8], int win_lo, unsigned long long N, double h1, int& status, double& arg,
                         long long* tl) {
    static_assert(kHistBins == 8 * 64, "eight histogram bins per lane");
    const uint32_t lane = threadIdx.x & 63u;
    // the log-Weibull fit sees only the samples a sampled record keeps: the
    // histogram restricted to its window (zero outside)
    int32_t hv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) hv[i] = h[i];
    if constexpr (FIT == PS_FIT_GUMBEL) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = 8 * (int)lane + i;
            if (hv[i] < 0 || win_lo < 0 || j < win_lo || j >= win_lo + PS_SAMPLE_BINS) hv[i] = 0;
        }
    }
    const int32_t lm2 = __shfl_up(hv[6], 1, 64), lm1 = __shfl_up(hv[7], 1, 64);
    const int32_t rp0 = __shfl_down(hv[0], 1, 64), rp1 = __shfl_down(hv[1], 1, 64);
    int32_t x[12];
    x[0] = lane ? lm2 : 0;
    x[1] = lane ? lm1 : 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i + 2] = hv[i];
    x[10] = lane < 63u ? rp0 : 0;
    x[11] = lane < 63u ? rp1 : 0;
    long long num[8];
    long long lt = 0;
    unsigned long long key = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        long long acc = 0;
        if (N) acc = -3ll * x[i] + 12ll * x[i + 1] + 17ll * x[i + 2] + 12ll * x[i + 3] - 3ll * x[i + 4];
        num[i] = acc < 0 ? 0 : acc;
        lt += num[i];
        // mode: largest numerator, lowest bin on ties -> max of (value << 9 | (511 - j))
        const unsigned long long kk = ((unsigned long long)num[i] << 9) |
                                      (unsigned long long)(kHistBins - 1 - (int)(8u * lane + i));
        key = kk > key ? kk : key;
    }
    key = wave_max_u64(key);
    const long long total = wave_sum_i64(lt);
    const int mode = kHistBins - 1 - (int)(key & 511ull);
    // smoothed mass of the lanes above this one: a suffix sum across lanes
    long long suf = lt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long v = __shfl_down(suf, o, 64);
        if (lane + (uint32_t)o < 64u) suf += v;
    }
    const long long above = suf - lt;
    arg = __builtin_nan("");
    if constexpr (FIT == PS_FIT_GUMBEL) {
        if (status != PS_STATUS_OK) return;                 // uniform across the wavefront
        if (total <= 0) { status = PS_STATUS_FEW_POINTS; return; }
        double wx = 0, pts = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            wx += (double)num[i] * (0.1 * (double)(8 * (int)lane + i) + 0.05);
            pts += num[i] > 0 ? 1.0 : 0.0;
        }
        const double m = wave_sum_f64(wx) / (double)total;
        const double n_pts = wave_sum_f64(pts);
        double d2 = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const double d = (0.1 * (double)(8 * (int)lane + i) + 0.05) - m;
            d2 += (double)num[i] * d * d;
        }
        const double sd2 = wave_sum_f64(d2);
        if (n_pts < 3.0) {
            status = PS_STATUS_FEW_POINTS;
        } else {
            const double v = sd2 / (double)total;
            const double beta = sqrt(6.0 * v) / 3.14159265358979323846;
            const double mu = m - 0.57721566490153286061 * beta;
            arg = (h1 - mu) / beta;
        }
        return;
    }
    // least-squares fit of log10 survival over [mode, bin(H1) - 1]
    double sx = 0, sy = 0, sxx = 0, sxy = 0, cnt = 0;
    if (status == PS_STATUS_OK && total > 0) {
        const double hb = floor(10.0 * h1);
        const int jh = hb >= (double)(kHistBins - 1) ? kHistBins - 1 : (int)hb;
        long long tail = above;
#pragma unroll
        for (int i = 7; i >= 0; --i) {
            tail += num[i];
            tl[64 * i + lane] = tail;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // every lane's sums are visible to the wave
        // the fit range [mode, jh - 1] dealt out to consecutive lanes, so each
        // log10 is taken by as many lanes as there are bins left to fit
        for (int j = mode + (int)lane; j <= jh - 1; j += 64) {
            const long long tj = tl[64 * (j & 7) + (j >> 3)];
            if (tj <= 0) continue;
            const double xj = 0.1 * (double)j;
            const double yj = log10((double)tj / (double)total);
            sx += xj; sy += yj; sxx += xj * xj; sxy += xj * yj; cnt += 1.0;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // reads done before the area is written again
    }
    sx = wave_sum_f64(sx);
    sy = wave_sum_f64(sy);
    sxx = wave_sum_f64(sxx);
    sxy = wave_sum_f64(sxy);
    cnt = wave_sum_f64(cnt);
    if (status != PS_STATUS_OK) return;
    if (cnt < 3.0) {
        status = PS_STATUS_FEW_POINTS;
        return;
    }
    const double num_w = cnt * sxy - sx * sy;
    const double den = cnt * sxx - sx * sx;
    const double w = num_w / den;
    const double b = (sy - w * sx) / cnt;
    if (!(w < 0.0)) status = PS_STATUS_BAD_SLOPE;
    else arg = w * h1 + b;
}

// Lane l's eight bins of a 512-bin histogram in global memory (two 16-byte loads).
__device__ __forceinline__ void load_bins(const int32_t* hist, int32_t h[8]) {
    const int4* p = (const int4*)hist + 2u * (threadIdx.x & 63u);
    const int4 a = p[0], b = p[1];
    h[0] = a.x; h[1] = a.y; h[2] = a.z; h[3] = a.w; h[4] = b.x; h[5] = b.y; h[6] = b.z; h[7] = b.w;
}

__device__ __forceinline__ void store_bins(int32_t* hist, const int32_t h[8]) {
    int4* p = (int4*)hist + 2u * (threadIdx.x & 63u);
    p[0] = make_int4(h[0], h[1], h[2], h[3]);
    p[1] = make_int4(h[4], h[5], h[6], h[7]);
}

__device__ __forceinline__ void store_stat(ps_stat* out, unsigned long long n_window, unsigned long long N, double ev,
                                           int status) {
    ps_stat st;
    st.n_window = n_window;
    st.n_scored = N;
    st.evalue = ev;
    st.status = status;
    st.pad = 0;
    *out = st;
}

}  // namespace

// The expect values from the fitted arguments of hdr->n spectra (or n_cap when
// hdr is NULL); defined below.
static hipError_t launch_finish(ps_stat* stats, uint64_t n_cap, const BatchHdr* hdr, int32_t fit,
                                hipStream_t stream);

// ---------------------------------------------------------------------------
// merge: partial top-k -> hits; histogram -> smoothed survival -> fit -> e-value
// ---------------------------------------------------------------------------

struct MergeArgs {
    DevSpectra sp;
    KParams kp;
    Work w;
    uint32_t per_item;   // 1: partial lists per work item (spec_item0 ranges); 0: one per spectrum
};

template <int FIT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_merge(MergeArgs A) {
    __shared__ long long s_tail[kStatWaves][8 * 64];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t K = A.kp.top_k;
    const uint64_t n_batch = A.sp.hdr->n;
    for (uint64_t s = (uint64_t)blockIdx.x * kStatWaves + (threadIdx.x >> 6); s < n_batch;
         s += (uint64_t)gridDim.x * kStatWaves) {
        const SpecInfo inf = A.w.info[s];
        const bool invalid = (inf.flags & kFlagInvalid) != 0;
        const bool overflow = (inf.flags & kFlagOverflow) != 0;
        uint64_t i0 = s, i1 = s + 1;
        if (A.per_item) { i0 = A.w.spec_item0[s]; i1 = A.w.spec_item0[s + 1]; }
        const uint32_t L = (invalid || overflow) ? 0u : (uint32_t)(i1 - i0);
        const ps_hit* src = A.w.partial + i0 * K;
        int32_t h[8];
        load_bins(A.w.hist + s * (uint64_t)kHistBins, h);
        const int win = fit_window<FIT>(h);
        const uint32_t c = wave_top_k(L, K, [&](uint32_t x) { return hit_key(src[x].hyperscore, src[x].id, x); });
        ps_hit mine;
        if (c != 0xFFFFFFFFu) mine = src[c]; else empty_hit(mine);
        if (lane < K) A.w.hits[s * K + lane] = mine;
        const double h1 = __shfl(mine.hyperscore, 0, 64);
        const unsigned long long N = (invalid || overflow) ? 0ull : A.w.n_scored[s];
        int status = invalid ? PS_STATUS_INVALID : overflow ? PS_STATUS_OVERFLOW
                   : N == 0 ? PS_STATUS_NO_HITS : PS_STATUS_OK;
        double ev;
        fit_wave<FIT>(h, win, N, h1, status, ev, s_tail[threadIdx.x >> 6]);
        if (lane == 0) store_stat(A.w.stats + s, invalid ? 0ull : (unsigned long long)(inf.hi - inf.lo), N, ev, status);
    }
}

hipError_t launch_merge(const DevIndex&, const DevSpectra& sp, const KParams& kp, const Work& w, bool per_item,
                        hipStream_t stream) {
    if (sp.n == 0) return hipSuccess;
    MergeArgs a{sp, kp, w, per_item ? 1u : 0u};
    const uint64_t blocks = (sp.n + kStatWaves - 1) / kStatWaves;
    const uint32_t grid = (uint32_t)(blocks < (1u << 20) ? blocks : (1u << 20));
    if (kp.fit == PS_FIT_GUMBEL) hipLaunchKernelGGL(k_merge<PS_FIT_GUMBEL>, dim3(grid), dim3(kBlock), 0, stream, a);
    else hipLaunchKernelGGL(k_merge<PS_FIT_TAIL>, dim3(grid), dim3(kBlock), 0, stream, a);
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_finish(w.stats, sp.n, sp.hdr, kp.fit, stream);
}

// ---------------------------------------------------------------------------
// result assembly over database partitions (Superstep 4; Supplementary
// Algorithm 4): histogram addition, G-way top-k merge, expect value
// ---------------------------------------------------------------------------

struct AssembleArgs {
    ps_part parts[PS_MAX_SHARDS];
    uint32_t G, K;
    int32_t fit;
    uint32_t all_hist;   // every partition gives a full histogram
    uint64_t n;
    ps_hit* hits;
    ps_stat* stats;
    int32_t* hist;   // may be NULL
};

template <int FIT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_assemble(AssembleArgs A) {
    __shared__ long long s_tail[kStatWaves][8 * 64];
    const uint32_t lane = threadIdx.x & 63u, G = A.G, K = A.K;
    for (uint64_t s = (uint64_t)blockIdx.x * kStatWaves + (threadIdx.x >> 6); s < A.n;
         s += (uint64_t)gridDim.x * kStatWaves) {
        // counts and flags of the G partitions: lane g reads partition g
        unsigned long long scored = 0, window = 0;
        uint32_t flags = 0;
        if (lane < G) {
            const ps_stat st = A.parts[lane].stats[s];
            scored = st.n_scored;
            window = st.n_window;
            flags = (st.status == PS_STATUS_INVALID ? 1u : 0u) | (st.status == PS_STATUS_OVERFLOW ? 2u : 0u);
        }
        scored = wave_sum_u64(scored);
        window = wave_sum_u64(window);
        flags = wave_or_u32(flags);
        const bool invalid = (flags & 1u) != 0, overflow = (flags & 2u) != 0;
        // histogram addition: full partition histograms share bin 0 and add one to
        // one; a sampled one is shifted to its window [lo, lo + 120) first
        int32_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (A.all_hist) {
            // four partitions' bins requested together (a group past G repeats
            // partition G - 1 and adds nothing)
            for (uint32_t g0 = 0; g0 < G; g0 += 4) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {         // this lane's bins 4 at a time
                    int4 q[4];
#pragma unroll
                    for (uint32_t u = 0; u < 4; ++u)
                        q[u] = ((const int4*)(A.parts[min(g0 + u, G - 1)].hist + s * (uint64_t)kHistBins))
                            [2u * lane + (uint32_t)half];
#pragma unroll
                    for (uint32_t u = 0; u < 4; ++u) {
                        const bool in = g0 + u < G;
                        h[4 * half + 0] += in ? q[u].x : 0;
                        h[4 * half + 1] += in ? q[u].y : 0;
                        h[4 * half + 2] += in ? q[u].z : 0;
                        h[4 * half + 3] += in ? q[u].w : 0;
                    }
                }
            }
        } else for (uint32_t g = 0; g < G; ++g) {
            if (A.parts[g].hist) {
                int32_t v[8];
                load_bins(A.parts[g].hist + s * (uint64_t)kHistBins, v);
#pragma unroll
                for (int i = 0; i < 8; ++i) h[i] += v[i];
            } else {
                const ps_sampled* r = A.parts[g].sampled + s;
                const uint32_t lo = r->lo;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t j = 8u * lane + i - lo;   // wraps above 120 below the window
                    if (j < (uint32_t)PS_SAMPLE_BINS) h[i] += r->count[j];
                }
            }
        }
        if (A.hist) store_bins(A.hist + s * (uint64_t)kHistBins, h);
        const int win = fit_window<FIT>(h);
        // top-k of the partitions' lists, ids turned into whole-database ids
        const uint32_t c = wave_top_k((invalid || overflow) ? 0u : G, K, [&](uint32_t x) {
            const uint32_t g = x / K;
            const ps_hit& p = A.parts[g].hits[s * K + (x - g * K)];
            return hit_key(p.hyperscore, p.id == 0xFFFFFFFFu ? p.id : (uint32_t)((uint64_t)p.id * G + g), x);
        });
        ps_hit mine;
        if (c != 0xFFFFFFFFu) {
            const uint32_t g = c / K;
            mine = A.parts[g].hits[s * K + (c - g * K)];
            mine.id = (uint32_t)((uint64_t)mine.id * G + g);
        } else {
            empty_hit(mine);
        }
        if (lane < K) A.hits[s * K + lane] = mine;
        const double h1 = __shfl(mine.hyperscore, 0, 64);
        const unsigned long long N = (invalid || overflow) ? 0ull : scored;
        int status = invalid ? PS_STATUS_INVALID : overflow ? PS_STATUS_OVERFLOW
                   : N == 0 ? PS_STATUS_NO_HITS : PS_STATUS_OK;
        double ev;
        fit_wave<FIT>(h, win, N, h1, status, ev, s_tail[threadIdx.x >> 6]);
        if (lane == 0) store_stat(A.stats + s, invalid ? 0ull : window, N, ev, status);
    }
}

hipError_t launch_assemble(const ps_part* parts, uint32_t G, uint64_t n, uint32_t K, int32_t fit, ps_hit* hits,
                           ps_stat* stats, int32_t* hist, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    AssembleArgs a;
    memset(&a, 0, sizeof a);
    a.all_hist = 1;
    for (uint32_t g = 0; g < G; ++g) {
        a.parts[g] = parts[g];
        if (!parts[g].hist) a.all_hist = 0;
    }
    a.G = G; a.K = K; a.fit = fit; a.n = n; a.hits = hits; a.stats = stats; a.hist = hist;
    const uint64_t blocks = (n + kStatWaves - 1) / kStatWaves;
    const uint32_t grid = (uint32_t)(blocks < (1u << 20) ? blocks : (1u << 20));
    if (fit == PS_FIT_GUMBEL) hipLaunchKernelGGL(k_assemble<PS_FIT_GUMBEL>, dim3(grid), dim3(kBlock), 0, stream, a);
    else hipLaunchKernelGGL(k_assemble<PS_FIT_TAIL>, dim3(grid), dim3(kBlock), 0, stream, a);
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_finish(stats, n, nullptr, fit, stream);
}

// ---------------------------------------------------------------------------
// expect values from the fitted arguments (one thread per spectrum)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_finish_evalue(ps_stat* stats, uint64_t n_cap, const BatchHdr* hdr,
                                                          int32_t fit) {
    const uint64_t n = hdr ? hdr->n : n_cap;
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < n; s += (uint64_t)gridDim.x * blockDim.x) {
        ps_stat st = stats[s];
        if (st.status != PS_STATUS_OK) continue;
        const double N = (double)st.n_scored, arg = st.evalue;
        st.evalue = fit == PS_FIT_GUMBEL ? N * -expm1(-exp(-arg)) : N * pow(10.0, arg);
        stats[s].evalue = st.evalue;
    }
}

static hipError_t launch_finish(ps_stat* stats, uint64_t n_cap, const BatchHdr* hdr, int32_t fit,
                                hipStream_t stream) {
    const uint64_t blocks = (n_cap + kBlock - 1) / kBlock;
    const uint32_t grid = (uint32_t)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_finish_evalue, dim3(grid), dim3(kBlock), 0, stream, stats, n_cap, hdr, fit);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sampling: one wavefront per spectrum turns its 512-bin histogram into the
// 256-byte record of the Sampling section
// ---------------------------------------------------------------------------

struct SampleArgs {
    const int32_t* hist;
    const ps_stat* stats;
    ps_sampled* out;
    uint64_t n;
};

constexpr uint32_t kSampleWaves = kBlock / 64;

__global__ __launch_bounds__(kBlock) void k_sample(SampleArgs A) {
    __shared__ int32_t s_h[kSampleWaves][kHistBins];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    int32_t* h = s_h[wave];
    for (uint64_t s = (uint64_t)blockIdx.x * kSampleWaves + wave; s < A.n; s += (uint64_t)gridDim.x * kSampleWaves) {
        // lane l holds bins 8 l .. 8 l + 7 (negative counts, which a search never
        // writes, count as empty)
        const int4* src = (const int4*)(A.hist + s * (uint64_t)kHistBins) + 2u * lane;
        const int4 a = src[0], b = src[1];
        int32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            v[i] = v[i] > 0 ? v[i] : 0;
            h[8u * lane + i] = v[i];
        }
        int lo = sample_window_lo(v);
        if (lo < 0) lo = 0;                                         // an empty histogram keeps nothing
        // flags from this lane's bins
        bool sat = false, lost = false;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = (int)(8u * lane) + i;
            const bool inside = j >= lo && j < lo + PS_SAMPLE_BINS;
            sat |= inside && v[i] > 65535;
            lost |= !inside && v[i] > 0;
        }
        const uint32_t flags = (__ballot(sat) ? 1u : 0u) | (__ballot(lost) ? 2u : 0u);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // the wave's LDS writes are visible to it
        // 64 words of the record: header, then count pairs
        uint32_t word;
        if (lane == 0) {
            word = (uint32_t)lo | (flags << 16);
        } else if (lane == 1) {
            word = 0;
        } else if (lane < 4) {
            const uint64_t ns = A.stats[s].n_scored;
            word = lane == 2 ? (uint32_t)ns : (uint32_t)(ns >> 32);
        } else {
            const int i = 2 * (int)(lane - 4);
            const int32_t c0 = h[lo + i], c1 = h[lo + i + 1];
            word = (uint32_t)min(c0, 65535) | ((uint32_t)min(c1, 65535) << 16);
        }
        ((uint32_t*)(A.out + s))[lane] = word;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // reads done before the next spectrum's writes
    }
}

hipError_t launch_sample(const int32_t* hist, const ps_stat* stats, ps_sampled* out, uint64_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    SampleArgs a{hist, stats, out, n};
    const uint64_t blocks = (n + kSampleWaves - 1) / kSampleWaves;
    const uint32_t grid = (uint32_t)(blocks < (1u << 20) ? blocks : (1u << 20));
    hipLaunchKernelGGL(k_sample, dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}


}  // namespace ps

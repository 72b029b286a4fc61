// internal.h -- shared definitions of the pepscan library (host code and kernels).
//
// Not part of the public ABI (include/pepscan.h is).  Units: integer
// micro-Dalton (uDa) masses; fragment bins of 10000 uDa rounded half up.
#pragma once
#include <stdint.h>
#include <stddef.h>

#include <hip/hip_runtime.h>

#include "pepscan.h"

namespace ps {

constexpr int64_t kProtonUda = 1007276;     // H+
constexpr int64_t kWaterUda = 18010565;     // H2O
constexpr int64_t kBinWidth = 10000;        // 0.01 Da
constexpr int64_t kCOUda = 27994915;        // CO, the a/b and x/y ion offset
constexpr int64_t kNH3Uda = 17026549;       // NH3, the c/b and z/y ion offset
constexpr int64_t kH2Uda = 2015650;         // H2

// Fragment ion series of an index, in posting order: N-terminal series first.
struct IonSeries {
    int n;                     // enabled series
    int64_t shift[6];          // added to b (N-terminal) or y (C-terminal) mass
    uint32_t cterm[6];         // 1: C-terminal (posting bit 1)
};
inline IonSeries ion_series(uint32_t types) {
    IonSeries s{};
    const uint32_t bit[6] = {PS_ION_A, PS_ION_B, PS_ION_C, PS_ION_X, PS_ION_Y, PS_ION_Z};
    const int64_t sh[6] = {-kCOUda, 0, kNH3Uda, kCOUda - kH2Uda, 0, -kNH3Uda};
    for (int t = 0; t < 6; ++t)
        if (types & bit[t]) { s.shift[s.n] = sh[t]; s.cterm[s.n] = t >= 3 ? 1u : 0u; ++s.n; }
    return s;
}
// Largest number of enabled series on one terminus.
inline uint32_t ion_mult(uint32_t types) {
    const uint32_t n = __builtin_popcount(types & (PS_ION_A | PS_ION_B | PS_ION_C));
    const uint32_t c = __builtin_popcount(types & (PS_ION_X | PS_ION_Y | PS_ION_Z));
    return n > c ? n : c;
}
constexpr int kHistBins = PS_HIST_BINS;
constexpr uint32_t kLfSize = 65536;         // log10(n!) table, n < 65536
constexpr uint32_t kLsSize = 1u << 20;      // log10(s) table, s < 2^20
constexpr uint32_t kEntryInvalid = 0xFFFFFFFFu;
constexpr uint32_t kPostPad = 0xFFFFFFFFu;  // filler after a list up to its quad boundary
// Postings are addressed as 16-byte quads with 32-bit indices: at most 2^32 quads.
constexpr uint64_t kMaxQuads = 1ull << 32;
constexpr int kBlock = 256;                 // threads per workgroup for every kernel
constexpr size_t kMaxLds = 156 * 1024;      // dynamic LDS per workgroup (160 KB on gfx950 less static use)

// Per-spectrum flags written by the prep kernel.
enum : uint32_t {
    kFlagInvalid = 1u,      // spectrum rejected (status PS_STATUS_INVALID)
    kFlagWide = 2u,         // needs 64-bit shared-peak counters
    kFlagOverflow = 4u,     // even 64-bit counters / tables cannot hold it
};

constexpr uint32_t kMaxDense = PS_MAX_DENSE;   // dense maps per index
static_assert(kMaxDense <= 8, "a dense table entry holds a 3-bit map slot");
constexpr uint64_t kDenseIdAlign = 32768;      // the largest tile: maps cover whole tiles
inline uint64_t dense_map_bytes(uint64_t n_pep) {
    return (n_pep + kDenseIdAlign - 1) / kDenseIdAlign * (kDenseIdAlign / 4);
}

// Device view of an uploaded index.
struct DevIndex {
    const int64_t* mass;       // [n_pep], ascending
    const uint32_t* bin_q;     // [n_bins + 1] bin b's list starts at posting 4 * bin_q[b] (lists are
                               // padded to whole 16-byte quads; the last entry is the quad count)
    const uint32_t* post;      // [4 * bin_q[n_bins]], value = id << 1 | is_y, sorted within a bin;
                               // padding entries are kPostPad and lie beyond every list's end
    const double* lf;          // [kLfSize]  lf[n] = sum_{k=2..n} log10 k
    const double* ls;          // [kLsSize]  ls[s] = log10 s
    const uint32_t* dir;       // [n_bins * dir_stride] first posting of a bin at or after each id
                               // block, as a position inside the bin's own list
    uint32_t dir_shift;        // id block = 1 << dir_shift ids (the tile grain)
    uint32_t dir_nblk;
    uint32_t dir_stride;       // row length, a multiple of 4 (rows are 16-byte aligned)
    uint32_t merge_tol;        // T > 0: the list of bin b holds bins b-T..b+T (one probe per peak)
    uint64_t n_pep, n_bins, n_post;
    uint32_t max_len;          // longest peptide (residues)
    uint32_t ion_mult;         // most ion series on one terminus (counter bounds)
    uint32_t ion_series;       // enabled ion series
    int64_t min_residue;       // lightest residue incl. modification deltas (uDa)
    // Dense lists: a list holding a large share of all ids is also kept as a
    // map of two bits per id.  Byte g of a map covers ids 4g..4g+3: bit e is
    // set when id 4g+e has a C-terminal posting in the list, bit 4+e when it
    // has an N-terminal one.  Maps are zero up to a multiple of kDenseIdAlign
    // ids, and a list becomes dense only if no (id, terminus) occurs twice in
    // it, so the map holds exactly the list's postings.
    // dense_tab[j] describes map j: bin | c << 24 | slot << 28, where c (1 or
    // 2) is the most a probe on the list adds to one id's count and the map
    // starts at dense_maps + slot * dense_stride.
    const uint32_t* dense_tab;
    const uint8_t* dense_maps;
    uint64_t dense_stride;
    uint32_t n_dense;          // maps in use (0: every list is scanned as postings)
};


// Per-spectrum summary written by the prep kernel.
struct SpecInfo {
    uint32_t lo, hi;           // window as id range [lo, hi)
    uint32_t n_ent;            // entry slots used (kept peaks x fragment charges)
    uint32_t flags;
};

// Actual size of the batch in flight, in device memory, so that one launch
// sequence (or one captured graph) serves any batch up to its capacity.
struct BatchHdr {
    unsigned long long n;      // spectra
    unsigned long long nnz;    // peaks (length of mz / inten)
};

// Inputs of one batch, device pointers.
struct DevSpectra {
    const uint64_t* peak_off;
    const float* mz;
    const float* inten;
    const double* prec;
    const int8_t* charge;
    uint64_t n;                // capacity: grids are sized for it
    uint64_t nnz;              // capacity
    const BatchHdr* hdr;       // actual n and nnz; peak_off entries beyond nnz are invalid
};

// Search settings as the kernels see them.
struct KParams {
    int64_t window;
    int32_t window_is_ppm;
    int32_t tol;               // T
    uint32_t top_peaks;        // B
    uint32_t top_k;
    uint32_t min_shared;
    uint32_t max_charge;
    uint32_t ent_stride;       // entry slots per spectrum = top_peaks * max(1, max_charge - 1)
    uint32_t seg_cap;          // probe slots per workgroup (entries x bin offsets)
    uint32_t tile;             // candidates per LDS counter tile: a power of two, >= 1 << dir_shift
    uint32_t tile_shift;       // log2(tile)
    uint32_t nt;               // threads per scan workgroup: 256 or 512 (tile >= 16 nt)
    int32_t fit;               // PS_FIT_TAIL or PS_FIT_GUMBEL
    uint32_t noise_permille;   // peaks below Imax * noise_permille / 1000 are dropped before top-B
    int32_t intensity;         // PS_INTENSITY_LINEAR or PS_INTENSITY_SQRT
};

// Workspace pointers of one batch (all inside the caller's device block).
struct Work {
    BatchHdr* hdr;             // actual batch size
    uint32_t* entries;         // [n * ent_stride] (bin << 8 | q) or kEntryInvalid
    SpecInfo* info;            // [n]
    int32_t* hist;             // [n * 512]
    unsigned long long* n_scored;  // [n]
    ps_hit* partial;           // [n_items * top_k]
    uint32_t* spec_item0;      // [n + 1] first item of each spectrum
    ps_hit* hits;              // [n * top_k]
    ps_stat* stats;            // [n]
    unsigned long long* counters;  // [kNumCounters], slots below
    // optional full dump of scored candidates
    uint32_t* dump_spec; uint32_t* dump_id; uint32_t* dump_cnt_lo; uint32_t* dump_cnt_hi;
    uint64_t dump_cap;
};

enum CounterSlot {
    kCtrPostings = 0, kCtrLookups = 1, kCtrQueue = 2, kCtrItems = 3, kCtrDump = 4,
    kCtrWide = 5,      // spectra that need 64-bit shared-peak counters
    kCtrOverflow = 6,  // spectra whose counter bound passes even the 64-bit form
    kCtrDensePost = 7, // postings counted through dense maps (included in kCtrPostings)
    kCtrDenseIds = 8,  // dense-map reads (candidates times dense probes)
};
constexpr uint32_t kNumCounters = 16;

// Launchers (kernels.hip).  All enqueue on `stream` and return the HIP status.
hipError_t launch_fill_u32(void* p, uint32_t value, uint64_t count, hipStream_t stream);
// write the actual batch size into a device header (a kernel, so it can be captured)
hipError_t launch_set_header(BatchHdr* hdr, uint64_t n, uint64_t nnz, hipStream_t stream);
// fill count_per_spectrum * hdr->n words (grid sized for `cap_count`)
hipError_t launch_fill_per_spectrum(void* p, uint32_t value, uint64_t count_per_spectrum, uint64_t cap_count,
                                    const BatchHdr* hdr, hipStream_t stream);
int device_cu_count();
hipError_t launch_prep(const DevIndex& ix, const DevSpectra& sp, const KParams& kp, const Work& w,
                       hipStream_t stream);
// per_item: partial lists are laid out per work item (persistent schedule);
// wide_only: launch only the 64-bit-counter kernel (the persistent kernel
// handles the narrow spectra)
hipError_t launch_scan_plain(const DevIndex& ix, const DevSpectra& sp, const KParams& kp, const Work& w,
                             bool dump, bool per_item, bool wide_only, hipStream_t stream);
hipError_t launch_worklist(const DevSpectra& sp, const KParams& kp, const Work& w, uint32_t tiles_per_item,
                           hipStream_t stream);
hipError_t launch_scan_persistent(const DevIndex& ix, const DevSpectra& sp, const KParams& kp,
                                  const Work& w, uint32_t grid, uint32_t tiles_per_item,
                                  hipStream_t stream);
hipError_t launch_merge(const DevIndex& ix, const DevSpectra& sp, const KParams& kp, const Work& w,
                        bool per_item, hipStream_t stream);
hipError_t launch_sample(const int32_t* hist, const ps_stat* stats, ps_sampled* out, uint64_t n, hipStream_t stream);
hipError_t launch_assemble(const ps_part* parts, uint32_t n_shards, uint64_t n, uint32_t top_k, int32_t fit, ps_hit* hits,
                           ps_stat* stats, int32_t* hist, hipStream_t stream);
size_t scan_lds_bytes(const KParams& kp, bool wide);
hipError_t init_kernel_attributes();

}  // namespace ps

/*
 * pepscan.h -- C ABI of the MI355X open-search library.
 *
 * The library searches MS/MS spectra against a fragment-ion index of a
 * digested, modified protein database, as the partial database search of
 * HiCOPS (arXiv 2102.02286, Superstep 3, Supplementary Algorithm 3) plus the
 * per-spectrum statistics of Superstep 4 (Supplementary Algorithm 4):
 *
 *   precursor-mass window  ->  per-peak fragment-bin postings  ->  shared-peak
 *   counts and intensity sums per candidate  ->  hyperscore  ->  top-k  ->
 *   score histogram  ->  smoothed survival function, tail fit, expect value.
 *
 * Every step after the index build runs in HIP kernels on one gfx950 GPU.
 * The index is built on the host or on the GPU (Superstep 1, Supplementary
 * Algorithm 1) and then lives in device memory the caller provides.
 *
 * Conventions (all entry points):
 *   - Return codes: PS_OK (0) or one of PS_E*.  Nothing throws across the ABI.
 *     ps_last_error() gives a thread-local message for the last failure.
 *   - Masses are integer micro-Dalton (uDa, 1e-6 Da) unless a name says
 *     otherwise.  Fragment bins are 0.01 Da (10000 uDa) wide, rounded half up:
 *     bin(m) = floor((m + 5000) / 10000).
 *   - Device memory: the library allocates no device memory, except the one
 *     static work area of ps_search_static.  Every other device buffer lives
 *     inside a caller-provided block (ps_device.base/bytes); the caller keeps
 *     it alive while any object built in it is in use.
 *   - Streams: work is enqueued on ps_device.stream (a hipStream_t, NULL = the
 *     null stream).  Calls are asynchronous unless a comment says "blocks".
 *   - Thread safety: an index is immutable after build and may be shared by
 *     concurrent searches; a batch or a server handle is used by one thread
 *     at a time unless stated.
 */
#ifndef PEPSCAN_H
#define PEPSCAN_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define PS_OK        0
#define PS_EINVAL    1   /* invalid argument; nothing was enqueued */
#define PS_ENOMEM    2   /* the caller's device block (or host memory) is too small */
#define PS_EAGAIN    3   /* admission refused for now (serving); retry later */
#define PS_EDEVICE   4   /* HIP error, or no usable gfx950 device */
#define PS_EOVERFLOW 5   /* a counter or table bound was exceeded (never silently saturated) */

/* ---- per-spectrum status (ps_stat.status) ------------------------------ */
#define PS_STATUS_OK          0  /* expect value computed */
#define PS_STATUS_NO_HITS     1  /* no candidate reached min_shared shared peaks */
#define PS_STATUS_FEW_POINTS  2  /* tail fit had fewer than 3 points (expect value NaN) */
#define PS_STATUS_BAD_SLOPE   3  /* fitted survival slope >= 0 (expect value NaN) */
#define PS_STATUS_INVALID     4  /* invalid spectrum (charge, peaks, precursor or limits) */
#define PS_STATUS_OVERFLOW    5  /* a shared-peak counter bound was exceeded */

#define PS_HIST_BINS 512         /* score histogram: 512 x int32 = 2048 bytes per spectrum */
#define PS_MAX_TOP_K 16
#define PS_MAX_TOP_PEAKS 256
#define PS_MAX_CHARGE 8
#define PS_MAX_FRAG_TOL_BINS 4
#define PS_MAX_PEAKS_IN 4096     /* input peaks per spectrum before top-B selection */
#define PS_MAX_SEGMENTS 2048     /* top_peaks * max(1, z-1) * probes per peak (2T+1, or 1 on an
                                    index with merged lists) per spectrum */

#define PS_ION_A 1u               /* a = b - CO */
#define PS_ION_B 2u
#define PS_ION_C 4u               /* c = b + NH3 */
#define PS_ION_X 8u               /* x = y + CO - H2 */
#define PS_ION_Y 16u
#define PS_ION_Z 32u              /* z = y - NH3 */

#define PS_MAX_SHARDS 64          /* database partitions one ps_assemble call merges */
#define PS_SAMPLE_BINS 120        /* histogram bins a sampled partial result keeps (Sampling: s = 120) */
#define PS_SAMPLE_HEAD 60         /* bins below the mean a sampled result keeps at most */

#define PS_FIT_TAIL   0          /* linear fit of the log survival function's tail (Superstep 4) */
#define PS_FIT_GUMBEL 1          /* log-Weibull (Gumbel) fit by moments (Superstep 4) */

#define PS_INTENSITY_LINEAR 0
#define PS_INTENSITY_SQRT   1

#define PS_SCHED_PLAIN      0    /* one workgroup per spectrum, separate launches */
#define PS_SCHED_PERSISTENT 1    /* one persistent work-queue launch (hipGraph) */

typedef struct ps_index  ps_index;
typedef struct ps_batch  ps_batch;
typedef struct ps_server ps_server;

/* A caller-owned block of device memory and the stream to work on. */
typedef struct {
    void*    base;        /* device pointer, 256-byte aligned */
    uint64_t bytes;
    void*    stream;      /* hipStream_t; NULL = null stream */
} ps_device;

/* A variable modification (Experimental Setup: "the number and type of PTMs
 * ... were varied").  Each residue letter may appear in at most one mod, and at
 * most one mod may be an N-terminal one; each site carries at most one mod. */
typedef struct {
    const char* residues;      /* letters it may sit on, e.g. "STY"; ignored when nterm */
    int32_t     nterm;         /* 1: protein N-terminus only */
    int32_t     pad;
    int64_t     delta_udalton; /* mass shift, uDa */
} ps_mod;

/* In-silico digestion (Experimental Setup: trypsin, missed cleavages, length
 * range).  Trypsin cuts after K or R unless the next residue is P. */
typedef struct {
    uint32_t      missed_cleavages;
    uint32_t      min_len, max_len;   /* 2 <= min_len <= max_len <= 62 */
    uint32_t      n_mods;             /* <= 16 */
    uint32_t      max_mods;           /* modified sites per peptide */
    uint32_t      merge_tol_bins;     /* 0: one posting list per fragment bin.  T in 1..PS_MAX_FRAG_TOL_BINS:
                                         the list of bin b holds the postings of bins b-T..b+T, so a
                                         search probes one list per peak instead of 2T+1 (same pairs,
                                         Supplementary Text 4); searches on such an index must use
                                         frag_tol_bins == T (else PS_EINVAL).  Postings grow (2T+1)-fold. */
    uint32_t      n_shards;           /* database partitions G, 1..PS_MAX_SHARDS (0 means 1: the whole database) */
    uint32_t      shard;              /* this index's partition g < G.  The sorted database is scattered round
                                         robin (Superstep 1's is_mine, Supplementary Fig. 3): partition g holds
                                         the entries of whole-database rank r with r % G == g, in order, so its
                                         id i is whole-database id i * G + g.  Searches of a partition report
                                         partition ids; ps_assemble turns G partition results into whole ones. */
    uint32_t      ion_types;          /* fragment ion series indexed, PS_ION_* bits; 0 = b and y (the paper's
                                         choice; its Mod Distance text says a, c, x, z generalise).  Matches of
                                         N-terminal series (a, b, c) count in n_b, C-terminal (x, y, z) in n_y.
                                         With a or x ions every residue must weigh more than 28.05 Da. */
    uint32_t      reserved;           /* must be 0 */
    const ps_mod* mods;
} ps_db_params;

/* A batch of spectra in CSR form (host or device pointers, see each call).
 * Spectrum i has peaks [peak_off[i], peak_off[i+1]); m/z and intensity are
 * float32, the precursor m/z float64, the precursor charge int8 in [1, 8]. */
typedef struct {
    uint64_t        n;
    const uint64_t* peak_off;      /* n + 1 */
    const float*    mz;
    const float*    intensity;
    const double*   precursor_mz;
    const int8_t*   charge;
} ps_spectra;

typedef struct {
    int32_t  window_is_ppm;   /* 1: `window` in ppm of the precursor mass; 0: uDa */
    int32_t  frag_tol_bins;   /* T: a peak matches an ion when |bin difference| <= T */
    int64_t  window;          /* precursor tolerance: |M_pep - M_q| <= window (inclusive) */
    uint32_t top_peaks;       /* B most intense peaks kept per spectrum */
    uint32_t top_k;           /* hits reported per spectrum, 1..PS_MAX_TOP_K */
    uint32_t min_shared;      /* k_min: candidates need >= k_min shared peaks to be scored */
    uint32_t max_charge;      /* largest precursor charge in the batch, 1..PS_MAX_CHARGE; sizes
                                 the workspace (fragment charges 1..max(1, z-1) per spectrum) */
    int32_t  schedule;        /* PS_SCHED_PLAIN or PS_SCHED_PERSISTENT */
    int32_t  want_hist;       /* 1: keep per-spectrum histograms for ps_results */
    int32_t  fit;             /* expect-value model on the smoothed histogram (Superstep 4 names both):
                                 PS_FIT_TAIL: least-squares line through log10 of the survival function
                                 from the mode to the bin below the top hit, ev = N * 10^(w H1 + b);
                                 PS_FIT_GUMBEL: Gumbel location and scale from the mean and variance of
                                 the histogram (bin centres 0.1 j + 0.05), ev = N * S(H1) with
                                 S(h) = 1 - exp(-exp(-(h - mu) / beta)); fewer than 3 non-zero smoothed
                                 bins gives PS_STATUS_FEW_POINTS */
    uint32_t noise_permille;  /* pre-processing (Superstep 2 names noise clearing): peaks with
                                 I < Imax * noise_permille / 1000 are dropped before the top-B
                                 selection; 0..1000, 0 keeps every peak */
    int32_t  intensity;       /* integer intensities q in [1, 100] relative to the most intense peak:
                                 PS_INTENSITY_LINEAR q = round half up of 100 I / Imax;
                                 PS_INTENSITY_SQRT q = the largest k with (k - 1/2)^2 <= 10^4 I / Imax
                                 (round half up of 100 sqrt(I / Imax), decided in fp64) */
    int32_t  reserved;        /* must be 0 */
} ps_search_params;

/* One reported candidate.  id = rank of the peptide in the index's sort order
 * (mass, protein, start, length, site mask).  Empty slots: id = UINT32_MAX,
 * hyperscore = -inf. */
typedef struct {
    uint32_t id;
    uint16_t n_b, n_y;        /* shared b- and y-ion pairs */
    uint32_t sum_q;           /* sum of matched peak intensities (integer 1..100 scale) */
    uint32_t pad;
    double   hyperscore;      /* log10(n_b! * n_y! * sum_q) */
} ps_hit;

typedef struct {
    uint64_t n_window;        /* candidates in the precursor window */
    uint64_t n_scored;        /* candidates with >= min_shared shared peaks */
    double   evalue;          /* expect value of the top hit, NaN unless status == OK */
    int32_t  status;          /* PS_STATUS_* */
    int32_t  pad;
} ps_stat;

/* Launch schedule of the posting scan.  Every schedule gives identical results;
 * it only changes speed.  Chosen by default at index creation, by ps_autotune,
 * or set by the caller. */
typedef struct {
    uint32_t tile;            /* candidates per LDS counter tile: a power of two in 1024..32768 and
                                 at least the index's tile grain (ps_index_directory) */
    uint32_t tiles_per_item;  /* PS_SCHED_PERSISTENT: tiles per work item (1..4096) */
    uint32_t groups_per_cu;   /* PS_SCHED_PERSISTENT: resident workgroups per compute unit (1..8) */
    uint32_t group_threads;   /* threads per scan workgroup sharing one tile of counters: 256 (0 means
                                 256) or 512; 512 needs tiles of at least 8192 candidates */
    uint32_t reserved[2];     /* must be 0 */
} ps_schedule;

/* ---- errors ------------------------------------------------------------ */
const char* ps_last_error(void);

/* ---- index ------------------------------------------------------------- */

/* Digest the proteins (residues concatenated, protein i = residues[prot_off[i],
 * prot_off[i+1])), enumerate modified forms, sort them by (mass, protein,
 * start, length, site mask) and build the CSR fragment-ion index (b/y ions at
 * charge 1) in host memory (Superstep 1; Supplementary Algorithm 1).  Inputs
 * are copied; the caller keeps ownership.  Only the 20 standard residue letters
 * are accepted (PS_EINVAL otherwise).  Needs no GPU. */
int ps_index_create(const ps_db_params* params, const char* residues, const uint64_t* prot_off,
                    uint64_t n_proteins, ps_index** out);

/* Device bytes the index needs (masses, bin offsets, postings, score tables). */
int ps_index_device_bytes(const ps_index* idx, uint64_t* bytes);

/* Copy the index into dev->base (which must hold ps_index_device_bytes) on
 * dev->stream.  Blocks until the copy is done.  PS_ENOMEM if the block is too
 * small; PS_EDEVICE without a usable device. */
int ps_index_upload(ps_index* idx, const ps_device* dev);

/* ps_index_create + ps_index_upload. */
int ps_build_index(const ps_device* dev, const ps_db_params* params, const char* residues,
                   const uint64_t* prot_off, uint64_t n_proteins, ps_index** out);

/* Sizes: peptides (database entries), postings, fragment bins. */
int ps_index_shape(const ps_index* idx, uint64_t* n_peptides, uint64_t* n_postings, uint64_t* n_bins);

/* The same index built on the GPU (Superstep 1; Supplementary Algorithm 1): the
 * host only counts each protein's entries (binomial sums over modification
 * sites); the GPU writes the entries, sorts them by mass (stable radix sort, so
 * ties keep the (protein, start, length, site mask) order), generates the b/y
 * ions and fills the CSR lists with a counting sort done in chunks of at most
 * chunk_pairs_cap (bin, posting) pairs (0: 2^29; a chunk always holds at least
 * one peptide's postings), then the tile directory.  More than one chunk costs
 * a second pass over the pairs but bounds the scratch memory.  The result is identical
 * to ps_index_create + ps_index_upload (every array bit for bit), already on the
 * device.  Its postings, directory and entry table stay on the device (the host
 * keeps the proteins and the bin offsets): ps_index_host_arrays,
 * ps_index_directory, ps_index_entry, ps_index_entries and ps_peptide copy what
 * they need back on request, blocking.
 *
 * ps_index_build_device_bytes: device bytes of the index block (kept for the
 * index's lifetime: masses, entry table, postings sized to an upper bound that
 * is exact for a whole database and, for a partition, its entries times the
 * longest peptide's postings, directory) and of the scratch block (only during
 * the build).  Needs a device
 * (it sizes the library sorts' workspace).
 * ps_index_build_device: builds into `index_block` (256-byte aligned) using
 * `scratch`; blocks until done, on index_block->stream.  Errors as
 * ps_index_create, plus PS_ENOMEM when a block is too small. */
int ps_index_build_device_bytes(const ps_db_params* params, const char* residues, const uint64_t* prot_off,
                                uint64_t n_proteins, uint64_t chunk_pairs_cap, uint64_t* index_bytes,
                                uint64_t* scratch_bytes);
int ps_index_build_device(const ps_db_params* params, const char* residues, const uint64_t* prot_off,
                          uint64_t n_proteins, uint64_t chunk_pairs_cap, const ps_device* index_block,
                          const ps_device* scratch, ps_index** out);

/* Entry `id`: mass (uDa), protein, start, length, site mask.  Mask bit i is
 * the i-th modifiable site, the protein N-terminus first, then residues by
 * position. */
int ps_index_entry(const ps_index* idx, uint64_t id, int64_t* mass, uint32_t* protein,
                   uint32_t* start, uint32_t* length, uint64_t* site_mask);

/* Entries [first, first + count) as arrays (any pointer may be NULL); ids past
 * the end are PS_EINVAL. */
int ps_index_entries(const ps_index* idx, uint64_t first, uint64_t count, int64_t* mass, uint32_t* protein,
                     uint32_t* start, uint8_t* length, uint64_t* site_mask);

/* Peptide string with modifications, e.g. "PEPT[+79.966331]IDEK"; PS_ENOMEM
 * if cap is too small (the string is truncated and NUL-terminated). */
int ps_peptide(const ps_index* idx, uint32_t id, char* buf, size_t cap);

/* Host copy of the CSR index, for checks: bin_off[n_bins + 1], postings[n]
 * (value = id << 1 | is_y, sorted within each bin). Either pointer may be NULL. */
int ps_index_host_arrays(const ps_index* idx, uint64_t* bin_off, uint32_t* postings);

/* Schedule used by later searches on this index (not by batches in flight).
 * PS_EINVAL for out-of-range fields. */
int ps_index_set_schedule(ps_index* idx, const ps_schedule* schedule);
int ps_index_get_schedule(const ps_index* idx, ps_schedule* schedule);

/* The tile directory: for every fragment bin and every block of
 * 2^grain_shift peptide ids, the position inside the bin's list of its first
 * posting at or after the block (Superstep 3's filter_2 reads a bin's postings
 * inside an id range; the directory turns every tile boundary of that range
 * into one load).  Positions are relative to the list's start, so they stay
 * 32-bit however many postings the index holds.  grain_shift is 12 unless the
 * directory would exceed 32 GiB; `bytes` is its size.  `dir`, if not NULL,
 * receives a host copy of `bytes` bytes laid out as [n_bins][stride] uint32
 * positions, stride = (n_pep >> grain_shift) + 2 rounded up to a multiple of 4
 * (the padding repeats the list's length).  Any pointer may be NULL. */
int ps_index_directory(const ps_index* idx, uint32_t* grain_shift, uint64_t* bytes, uint32_t* dir);

/* Dense lists.  Filter_2 of Superstep 3 counts, for every candidate in the
 * window, the fragment bins it shares with the spectrum.  A few bins are
 * shared by a large part of a tryptic database (the y1 ions of K and R hold
 * about half of all peptides each), so their lists are nearly as long as the
 * id range itself and take a large share of the scan.  Every list with at
 * least n_pep / 4 postings (the longest PS_MAX_DENSE) also gets a map of two
 * bits per peptide id on the device: one for a C-terminal (y-like) and one
 * for an N-terminal (b-like) posting of that id.  A probe on such a list is
 * then not streamed: the candidate filter admits every id whose other shared
 * peaks reach min_shared less the most the map probes could add, and each
 * admitted candidate reads its bits from the maps before it is scored or
 * dropped.  Results are identical either way.  Map probes are used only while
 * that lowered threshold stays at 2 or more (so with min_shared >= 3), at most
 * four per work item; others are streamed.  A list in which an (id, terminus)
 * pair repeats, or whose bin is 2^24 or above, keeps no map.  The maps cost
 * ceil(n_pep / 32768) * 8192 bytes each, in the index block.
 *
 * ps_index_dense: the number of maps (n_dense) and their bins (bins, room for
 * PS_MAX_DENSE, may be NULL); `enabled` says whether searches use them.
 * ps_index_set_dense: 0 makes later searches (and plans created afterwards)
 * stream every list, nonzero uses the maps again.  PS_EINVAL for NULL. */
#define PS_MAX_DENSE 8
int ps_index_dense(const ps_index* idx, uint32_t* n_dense, uint32_t* bins, int* enabled);
int ps_index_set_dense(ps_index* idx, int enabled);

void ps_index_free(ps_index* idx);

/* ---- one batch --------------------------------------------------------- */

/* Device bytes a batch of n spectra with nnz peaks needs in its workspace,
 * including a copy of the inputs (the buffers of Superstep 3's search and
 * Superstep 4's per-spectrum statistics). */
int ps_workspace_bytes(const ps_index* idx, uint64_t n, uint64_t nnz, const ps_search_params* params,
                       uint64_t* bytes);

/* Search host spectra: the partial database search of Superstep 3
 * (Supplementary Algorithm 3: pre-processing, precursor window, fragment-bin
 * postings, shared peaks, hyperscore, top-k, score histogram) followed by the
 * expect value of Superstep 4 (Supplementary Algorithm 4).  Validates the
 * spectra (PS_EINVAL on any invalid spectrum or parameter), copies them into
 * `work` (which must hold ps_workspace_bytes) and enqueues the whole search
 * on work->stream; returns without waiting. */
int ps_search_batch(ps_index* idx, const ps_device* work, const ps_spectra* spectra,
                    const ps_search_params* params, ps_batch** out);

/* The same search (Superstep 3 and Superstep 4's statistics) over spectra
 * already in device memory (every pointer of `spectra` is a device pointer),
 * as the GPU analogue of the paper's pre-loaded spectrum batches (Superstep 3,
 * Buffering).  Invalid spectra are reported per spectrum
 * (PS_STATUS_INVALID) instead of rejected.  Enqueues on work->stream and
 * returns without waiting; the inputs must stay valid until ps_results. */
int ps_search_device(ps_index* idx, const ps_device* work, const ps_spectra* spectra,
                     uint64_t nnz, const ps_search_params* params, ps_batch** out);

/* The per-spectrum results of Superstep 4: the best matches with their shared
 * peaks, intensity sums and hyperscores, the number of candidates scored, the
 * expect value of the top match and, optionally, the score histogram behind it
 * (2048 bytes per spectrum, the size the Sampling section gives).  Blocks until
 * the batch is done, then writes hits[n * top_k], stats[n] and, when the batch
 * was made with want_hist, hist[n * 512] (hist may be NULL).  Returns
 * PS_EOVERFLOW if any spectrum has PS_STATUS_OVERFLOW (results for the other
 * spectra are still written). */
int ps_results(ps_batch* batch, ps_hit* hits, ps_stat* stats, int32_t* hist);

/* Device pointers of the batch's results inside its workspace, laid out as
 * ps_results writes them: hits[n * top_k], stats[n], hist[n * 512] (the
 * histogram is always kept on the device, whatever want_hist says).  They are
 * written by the batch's work on its stream, stay valid while the batch and its
 * device block live, and are the inputs ps_assemble takes.  Any argument may be
 * NULL. */
int ps_batch_device_results(ps_batch* batch, ps_hit** hits, ps_stat** stats, int32_t** hist);

/* Every scored candidate (>= min_shared shared peaks) of every spectrum of a
 * finished batch, as (spectrum, id, packed counts).  Only for batches searched
 * with PS_SCHED_PLAIN and `dump` support (ps_search_dump); for parity checks. */
int ps_search_dump(ps_index* idx, const ps_device* work, const ps_spectra* spectra,
                   const ps_search_params* params, uint64_t cap, uint32_t* spectrum,
                   uint32_t* id, uint16_t* n_b, uint16_t* n_y, uint32_t* sum_q, uint64_t* count);

/* Device time of the last batch's dominant kernel (the posting scan), measured
 * with HIP events on the batch's stream: total milliseconds and launches.  Also
 * the number of postings it streamed (= sum over window candidates of shared
 * pairs) and of fragment-bin lookups it made. */
int ps_batch_timing(ps_batch* batch, double* scan_ms, uint32_t* scan_launches, uint64_t* postings,
                    uint64_t* bin_lookups);

/* Work counters of a finished search (of a batch, or of a plan's last run). */
typedef struct {
    uint64_t postings;          /* postings streamed = sum over window candidates of shared pairs */
    uint64_t bin_lookups;       /* fragment-bin lookups (probes with a bin inside the index) */
    uint64_t work_items;        /* persistent work items (0 for the plain schedule) */
    uint64_t wide_spectra;      /* spectra whose counter bound needs the 64-bit counters */
    uint64_t overflow_spectra;  /* spectra reported PS_STATUS_OVERFLOW */
    uint64_t dense_postings;    /* of `postings`, those counted through dense maps (ps_index_dense) */
    uint64_t dense_reads;       /* dense-map reads: candidates times dense probes */
    uint64_t reserved[1];
} ps_counters;

/* Blocks until the batch is done, then writes its counters.  PS_EINVAL for NULL. */
int ps_batch_counters(ps_batch* batch, ps_counters* out);

void ps_batch_free(ps_batch* batch);

/* ---- one batch without allocations -------------------------------------- */

/* Device bytes of the work area ps_search_static uses on each GPU. */
#define PS_STATIC_SCRATCH_BYTES (256ull << 20)

/* For callers that cannot allocate: code being captured into a hipGraph, tight
 * serving loops, harnesses that forbid allocation.  The same search as
 * ps_search_device (the same kernels, results equal bit for bit), enqueued on
 * `stream` (a hipStream_t, NULL = null stream).  Every pointer is device
 * memory the caller owns: the spectra (CSR with nnz peaks; they must stay valid
 * until the stream reaches the end of the search), and the outputs hits[n *
 * top_k], stats[n] and, when not NULL, hist[n * 512], which the kernels write
 * directly (nothing is copied to the host).  Every other buffer of the search
 * lives in one static work area of PS_STATIC_SCRATCH_BYTES that each GPU holds
 * from its first call until the process ends.  The call allocates nothing: no
 * device memory, no pinned host memory, no events, no host-to-device copy.
 * Calls that overlap on one GPU share that area and race: serialise them (one
 * stream, or wait for one call before the next).  Returns without waiting.
 * Errors: PS_EINVAL (NULL pointer, bad parameters, index not on the device),
 * PS_ENOMEM when the batch needs more than the static area (split the batch;
 * about 10k spectra of 200 peaks fit on a 40M-peptide index), PS_EDEVICE.
 * Invalid spectra are reported per spectrum (PS_STATUS_INVALID). */
int ps_search_static(ps_index* idx, void* stream, const ps_spectra* spectra, uint64_t nnz,
                     const ps_search_params* params, ps_hit* hits, ps_stat* stats, int32_t* hist);

/* ---- result assembly over database partitions --------------------------- */

/* Sampled partial histogram of one spectrum: the 256-byte intermediate result
 * of the Sampling section (Superstep 3) and its figure.  The histogram keeps
 * PS_SAMPLE_BINS consecutive bins [lo, lo + 120) around its mean, where the
 * mean is the average location (floored) of the three bins with the largest
 * counts (ties to the lower bin, nonzero bins only), and lo is the first
 * nonzero bin, or mean - PS_SAMPLE_HEAD when the head reaches further down, at
 * most 392 (the window ends by bin 511).  What does not fit is the far tail
 * first, which a fit recovers.  Counts above 65535 saturate. */
typedef struct {
    uint16_t lo;              /* histogram bin of count[0]; 0..392 */
    uint16_t flags;           /* bit 0: a count saturated; bit 1: a nonzero bin lay outside the window */
    uint32_t pad;             /* 0 */
    uint64_t n_scored;        /* the spectrum's scored candidates, all of them (ps_stat.n_scored) */
    uint16_t count[PS_SAMPLE_BINS];
} ps_sampled;                 /* 256 bytes */

/* Sample n partial histograms on the device (the Sampling section's step
 * before results leave a partition).  hist[n * 512] and stats[n] are a
 * search's device results (ps_batch_device_results, ps_plan_device_results);
 * out[n] is device memory.  Runs on `stream` (a hipStream_t, NULL = null
 * stream), allocates nothing and returns without waiting.  PS_EINVAL for a NULL
 * pointer when n > 0. */
int ps_sample(void* stream, uint64_t n, const int32_t* hist, const ps_stat* stats, ps_sampled* out);

/* The results of one partition's search (all device pointers, partition ids).
 * Exactly one of hist and sampled is given: the full histograms, or their
 * 256-byte samples from ps_sample. */
typedef struct {
    const ps_hit*     hits;      /* [n * top_k] */
    const ps_stat*    stats;     /* [n] */
    const int32_t*    hist;      /* [n * 512], or NULL */
    const ps_sampled* sampled;   /* [n], or NULL */
} ps_part;

/* Result assembly of Superstep 4 (Supplementary Algorithm 4) on the device.
 * parts[g] holds the results of the same n spectra searched with the same
 * parameters (top_k included) against partition g of G (ps_db_params.n_shards,
 * .shard).  Per spectrum, on `stream` (a hipStream_t, NULL = null stream):
 *   - hist = the sum of the partition histograms: full histograms add bin by
 *     bin; a sampled one is shifted to its window first (the "addition and
 *     shift" of Superstep 4), with zeros outside it;
 *   - hits = the best top_k of all partition hits by (hyperscore desc, id asc),
 *     ids turned into whole-database ids (i * G + g);
 *   - stats: n_window and n_scored are the sums; the expect value is fitted on
 *     the assembled histogram with the best hit's hyperscore, exactly as a search
 *     of the whole database does; a spectrum any partition reports INVALID or
 *     OVERFLOW keeps that status with no hits (n_scored 0).
 * With full histograms, or samples that lost nothing (flags 0), the result
 * equals a whole-database search bit for bit; lossy samples change only the
 * histogram and the expect value.  Outputs hits[n *
 * top_k], stats[n] and hist[n * 512] (hist may be NULL) are device memory that
 * must not overlap the inputs.  Nothing is allocated; returns without waiting.
 * PS_EINVAL for G outside 1..PS_MAX_SHARDS, top_k outside 1..PS_MAX_TOP_K, a
 * NULL input pointer when n > 0, or a partition giving both or neither of hist
 * and sampled.  `fit` is the ps_search_params.fit of the
 * partition searches. */
int ps_assemble(void* stream, uint32_t n_shards, const ps_part* parts, uint64_t n, uint32_t top_k, int32_t fit,
                ps_hit* hits, ps_stat* stats, int32_t* hist);

/* ---- reusable plans (persistent scan captured as a hipGraph) ------------ */

typedef struct ps_plan ps_plan;

/* Device bytes of a plan for batches of up to n_cap spectra and nnz_cap peaks. */
int ps_plan_bytes(const ps_index* idx, uint64_t n_cap, uint64_t nnz_cap, const ps_search_params* params,
                  uint64_t* bytes);

/* Carve a plan out of `work` (which must hold ps_plan_bytes) and capture the
 * whole kernel sequence of a search -- prep and window, work list, scan,
 * merge and expect values -- once as a hipGraph on work->stream (a private
 * non-blocking stream when NULL).  Every later run replays that graph; the
 * kernels read the batch size from device memory, so any batch up to the
 * capacity reuses it.  The index's current schedule is baked in. */
int ps_plan_create(ps_index* idx, const ps_device* work, uint64_t n_cap, uint64_t nnz_cap,
                   const ps_search_params* params, ps_plan** out);

/* Copy host spectra into the plan (validated as in ps_search_batch) and
 * replay the graph; returns without waiting.  Waits first if the plan's
 * previous run is still in flight (one batch per plan at a time). */
int ps_plan_run(ps_plan* plan, const ps_spectra* spectra);

/* Device pointers of the plan's input buffers (capacity n_cap / nnz_cap), for
 * callers that place spectra there themselves; then ps_plan_run_device. */
int ps_plan_inputs(ps_plan* plan, ps_spectra* device_buffers);
int ps_plan_run_device(ps_plan* plan, uint64_t n, uint64_t nnz);

/* Blocks until the run is done; then as ps_results. */
int ps_plan_results(ps_plan* plan, ps_hit* hits, ps_stat* stats, int32_t* hist);

/* Device time of the last run: the whole graph, and the scan alone (HIP events
 * recorded inside the graph; -1 when the runtime does not record them), plus
 * postings streamed, bin lookups and work items of the persistent scan. */
int ps_plan_timing(ps_plan* plan, double* graph_ms, double* scan_ms, uint64_t* postings, uint64_t* bin_lookups,
                   uint64_t* work_items);

/* Blocks until the plan's last run is done, then writes its counters (as
 * ps_batch_counters). */
int ps_plan_counters(ps_plan* plan, ps_counters* out);

/* Device pointers of the plan's results (as ps_batch_device_results), valid
 * for the last run once it is done on the plan's stream, until the next run. */
int ps_plan_device_results(ps_plan* plan, ps_hit** hits, ps_stat** stats, int32_t** hist);

/* The stream the plan runs on. */
int ps_plan_stream(ps_plan* plan, void** stream);

void ps_plan_free(ps_plan* plan);

/* ---- autotuning --------------------------------------------------------- */

typedef struct {
    ps_schedule schedule;
    double      scan_ms;     /* scan time on the sample (HIP events) */
    int32_t     same;        /* 1: results identical to the baseline schedule's */
    int32_t     pad;
} ps_tune_trial;

/* Choose the scan schedule for `params` by measurement: coordinate descent
 * over tile and, for PS_SCHED_PERSISTENT, tiles_per_item and groups_per_cu,
 * each candidate searching the host `sample` batch in `work` (candidates that do not fit it or the LDS are
 * skipped).  Every candidate's results must equal the starting schedule's bit
 * for bit (else PS_EDEVICE).  The fastest is set on the index and returned in
 * `best`.  With a cache_path, a schedule stored under the same index shape and
 * parameters is reused without measuring, and a new winner is written there.
 * `trials` (may be NULL) receives up to max_trials measured candidates. */
int ps_autotune(ps_index* idx, const ps_device* work, const ps_spectra* sample, const ps_search_params* params,
                const char* cache_path, ps_tune_trial* trials, uint32_t max_trials, uint32_t* n_trials,
                ps_schedule* best);

/* ---- serving: continuous batching over a resident index ----------------- */

typedef struct {
    uint64_t completed;       /* requests finished */
    uint64_t spectra;         /* spectra in finished requests */
    uint64_t runs;            /* device runs (each packs one or more requests) */
    uint64_t refused;         /* submissions refused with PS_EAGAIN */
    uint64_t max_queue;       /* deepest request queue seen */
    uint32_t streams;         /* concurrent device runs */
    uint32_t pad;
    uint64_t pool_bytes;      /* device bytes runs are admitted into */
    uint64_t peak_bytes;      /* most pool bytes reserved at once since the last reset */
    uint64_t committed_bytes; /* device bytes of the requests queued or running now */
    uint64_t samples;         /* latencies behind the percentiles */
    double   p50_ms, p99_ms, max_ms, mean_ms;   /* latency from submit to completion */
    double   elapsed_s;       /* first submit to last completion */
} ps_serve_stats;

/* A search server over an uploaded index (continuous batching; the paper's
 * analogue is Superstep 3's Buffering: a producer/consumer pipeline over
 * recycled buffers, and Supplementary Algorithm 5's memory guard).  The device
 * `pool` (256-byte aligned, owned by the caller, kept alive until
 * ps_server_free) is an arena: every run reserves exactly the workspace its
 * batch needs (as ps_workspace_bytes counts it) and gives it back when done.
 * A scheduler thread admits queued requests in arrival order: whenever one of
 * max_runs streams (1..64, each non-blocking at the default priority) is free,
 * it packs waiting requests into one run, up to run_spectra spectra and
 * run_peaks peaks (a single larger request runs alone), reserves the run's
 * bytes and enqueues the whole search.  So requests that arrive while others
 * run are admitted as streams and memory free up, and runs overlap on the
 * device.  A request that does not fit the free memory waits at the head of
 * the queue.  Memory guard: a submission is refused with PS_EAGAIN while the
 * device bytes of the queued and running requests plus its own would exceed
 * max_committed_bytes (0: the pool size).  params->schedule may be either
 * schedule.  Errors: PS_EINVAL (bad argument, index not on the device),
 * PS_ENOMEM (pool too small for a one-spectrum search), PS_EDEVICE. */
int ps_server_create(ps_index* idx, const ps_device* pool, const ps_search_params* params,
                     uint64_t run_spectra, uint64_t run_peaks, uint32_t max_runs, uint64_t max_committed_bytes,
                     ps_server** out);

/* Queue a request (host spectra, copied before returning).  Thread-safe.
 * PS_EAGAIN when the memory guard is closed (retry after requests finish; a
 * refused request leaves no trace), PS_ENOMEM when the request alone needs
 * more device bytes than the server holds, PS_EINVAL for invalid or empty
 * spectra.  *ticket identifies the request for ps_server_wait. */
int ps_server_submit(ps_server* server, const ps_spectra* spectra, uint64_t* ticket);

/* Block until the request is done; write its results as ps_results does and
 * its latency (submit to completion, ms).  Thread-safe; each ticket is waited
 * for by one caller: a second wait on a ticket already claimed, or an unknown
 * ticket, returns PS_EINVAL. */
int ps_server_wait(ps_server* server, uint64_t ticket, ps_hit* hits, ps_stat* stats, int32_t* hist,
                   double* latency_ms);

int ps_server_stats(ps_server* server, ps_serve_stats* out);
int ps_server_reset_stats(ps_server* server);

/* Drains queued and running requests, then frees the server (not the pool). */
void ps_server_free(ps_server* server);

#ifdef __cplusplus
}
#endif
#endif

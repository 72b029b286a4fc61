/*
 * oracle.h -- brute-force CPU reference for open-search database peptide search.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load or call this library.  The product
 * (the HIP library under paper_2102_02286_amd/) never links, loads or calls it,
 * and the two share no source, header, table or helper.
 *
 * What it computes (HiCOPS, arXiv 2102.02286):
 *   - peptide database: tryptic digestion with missed cleavages and a length
 *     range, variable modifications up to a per-peptide cap (Experimental Setup;
 *     database-size model D = zeta * 2^m in Notations; Supplementary Algorithm 1);
 *   - per spectrum: top-B most intense peaks (Superstep 3, sub-task R),
 *     precursor-mass filter (filter_1), shared-fragment-ion counting over b/y
 *     ions (filter_2; b/y only per the Superstep 1 footnote; shared peaks >= k
 *     per Supplementary Text 4), hyperscore, top hits (Supplementary Algorithm 3),
 *     a score histogram (Sampling section: the 2048-byte local null
 *     distribution), Savitzky-Golay smoothing, linear tail fit and expect value
 *     (Superstep 4; Supplementary Algorithm 4), or a log-Weibull (Gumbel) fit
 *     by moments in its place (Superstep 4 names both), over the samples the
 *     Sampling section keeps;
 *   - partitions and result assembly: round-robin database partitions and the
 *     histogram addition plus top-hit merge of Superstep 4 (Supplementary
 *     Algorithm 4).
 * Readings where the paper is silent are stated at each function in oracle.c.
 *
 * Everything floating-point is IEEE fp64; masses are exact int64 micro-Dalton.
 */
#ifndef PEPSCAN_ORACLE_H
#define PEPSCAN_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_HIST_BINS 512
#define ORC_MAX_MODS 16

typedef struct orc_db orc_db;

/* Database: proteins concatenated in `residues` with offsets `prot_off[n+1]`.
 * Modification j: residues given by bit (letter-'A') of mod_res_mask[j], or the
 * protein N-terminus when mod_nterm[j] != 0; mass delta mod_delta[j] (uDa).
 * `threads` worker threads digest and sort (the result does not depend on it).
 * Returns NULL on invalid input or when memory runs out. */
orc_db* orc_db_create(const char* residues, const uint64_t* prot_off, uint64_t n_prot,
                      uint32_t missed, uint32_t min_len, uint32_t max_len,
                      uint32_t n_mods, const uint32_t* mod_res_mask, const int32_t* mod_nterm,
                      const int64_t* mod_delta, uint32_t max_mods, int threads);
void     orc_db_free(orc_db*);
uint64_t orc_db_size(const orc_db*);
/* Peptide `id` (rank in the sorted key order): mass, protein, start, length, site mask. */
void     orc_db_get(const orc_db*, uint64_t id, int64_t* mass, uint32_t* prot,
                    uint32_t* start, uint32_t* len, uint64_t* mask);
/* Per-residue masses (uDa, modifications folded in) of peptide `id`; returns length. */
uint32_t orc_db_residue_masses(const orc_db*, uint64_t id, int64_t* out, uint32_t cap);

/* b_i and y_i, i = 1..n-1, of a residue-mass sequence (uDa). */
void orc_ions(const int64_t* res_uda, uint32_t n, int64_t* b_out, int64_t* y_out);

#define ORC_FIT_TAIL   0   /* linear tail fit of the log survival function */
#define ORC_FIT_GUMBEL 1   /* log-Weibull (Gumbel) fit */
#define ORC_ION_A 1u
#define ORC_ION_B 2u
#define ORC_ION_C 4u
#define ORC_ION_X 8u
#define ORC_ION_Y 16u
#define ORC_ION_Z 32u
#define ORC_INTENSITY_LINEAR 0   /* q = round(100 I / Imax) */
#define ORC_INTENSITY_SQRT   1   /* q = round(100 sqrt(I / Imax)) */

typedef struct {
    int32_t  window_is_ppm;   /* 1: window in ppm of the precursor mass; 0: uDa */
    int64_t  window;
    int32_t  frag_tol_bins;   /* T: |bin(peak) - bin(ion)| <= T */
    uint32_t top_peaks;       /* B */
    uint32_t top_k;           /* k <= 64 */
    uint32_t min_shared;      /* k_min */
    int32_t  fit;             /* ORC_FIT_TAIL or ORC_FIT_GUMBEL */
    uint32_t noise_permille;  /* peaks below this many thousandths of the most intense are dropped */
    int32_t  intensity;       /* ORC_INTENSITY_LINEAR or ORC_INTENSITY_SQRT */
    uint32_t ion_types;       /* ORC_ION_* bits; 0 means b and y */
} orc_params;

typedef struct {
    uint32_t id; uint16_t n_b, n_y; uint32_t sum_q; uint32_t pad; double hyperscore;
} orc_hit;

typedef struct {
    uint64_t n_window, n_scored;
    double   evalue;
    int32_t  status;          /* 0 ok, 1 no scored candidate, 2 < 3 fit points, 3 slope >= 0 */
    int32_t  pad;
    uint64_t lo, hi;          /* window as an id range [lo, hi) */
    uint64_t pairs_total;     /* sum over window candidates of shared pairs */
} orc_stat;

/* Search n spectra (host CSR) with `threads` worker threads.
 * hits[n*top_k], stats[n], hist[n*512] (hist may be NULL).  Returns 0, or -1 on
 * invalid input. */
int orc_search(const orc_db*, uint64_t n, const uint64_t* peak_off, const float* mz,
               const float* intensity, const double* precursor_mz, const int8_t* charge,
               const orc_params*, int threads, orc_hit* hits, orc_stat* stats, int32_t* hist);

/* Every scored candidate (pairs >= k_min) of one spectrum, in id order.
 * Returns the number found (entries written up to cap), or -1 on invalid input. */
int64_t orc_scored(const orc_db*, const uint64_t* peak_off_2, const float* mz,
                   const float* intensity, double precursor_mz, int8_t charge,
                   const orc_params*, uint32_t* ids, uint16_t* n_b, uint16_t* n_y,
                   uint32_t* sum_q, uint64_t cap);

/* Partition g of G: the entries whose rank r in the whole database has
 * r % G == g, in the same order (entry r is entry r / G of its partition).
 * Returns NULL when g >= G or G == 0. */
orc_db* orc_db_shard(const orc_db*, uint32_t n_shards, uint32_t shard);

/* Assemble the results of G partition searches of the same n spectra: inputs
 * part_hits[G][n][top_k] (partition-local ids), part_stats[G][n],
 * part_hist[G][n][512]; outputs as orc_search (global ids).  Returns 0, or -1
 * on invalid arguments. */
int orc_assemble(uint32_t n_shards, uint64_t n, uint32_t top_k, int32_t fit, const orc_hit* part_hits,
                 const orc_stat* part_stats, const int32_t* part_hist, orc_hit* hits,
                 orc_stat* stats, int32_t* hist);

/* Sampled intermediate result (Sampling section and its figure): the score
 * histogram cut to ORC_SAMPLE_BINS consecutive bins around its mean, so that
 * one spectrum's partial result fits 256 bytes.  Reading: the mean is the
 * average location (floored) of the three bins with the largest counts (ties:
 * lower bin; only nonzero bins); the window starts at the first nonzero bin,
 * or ORC_SAMPLE_HEAD bins below the mean if the head reaches further, so that
 * the far tail is what gets dropped first; it is clamped to end at bin 511.
 * Counts above 65535 saturate.  flags: bit 0 a count saturated, bit 1 a
 * nonzero bin fell outside the window. */
#define ORC_SAMPLE_BINS 120
#define ORC_SAMPLE_HEAD 60
typedef struct {
    uint16_t lo;               /* histogram bin of count[0] */
    uint16_t flags;
    uint32_t pad;
    uint64_t n_scored;         /* the spectrum's scored candidates (all of them) */
    uint16_t count[ORC_SAMPLE_BINS];
} orc_sampled;                 /* 256 bytes */

void orc_sample(const int32_t* hist, uint64_t n_scored, orc_sampled* out);
/* The shift of Superstep 4's "addition and shift": the 512-bin histogram a
 * record stands for (zero outside its window). */
void orc_unsample(const orc_sampled* in, int32_t* hist);

/* Pieces exposed for pin tests. */
double orc_hyperscore(uint32_t n_b, uint32_t n_y, uint32_t sum_q);
void   orc_sg_smooth(const int32_t* hist, double* out);          /* 512 -> 512 */
int    orc_evalue(const int32_t* hist, double top_h, uint64_t n_scored,
                  double* evalue, double* slope, double* intercept, int32_t* n_points);
int    orc_evalue_gumbel(const int32_t* hist, double top_h, uint64_t n_scored,
                         double* evalue, double* mu, double* beta, int32_t* n_points);

#ifdef __cplusplus
}
#endif
#endif

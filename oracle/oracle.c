/*
 * oracle.c -- plain, slow, brute-force CPU reference (see oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py; never by the product library.
 *
 * Method: HiCOPS (arXiv 2102.02286).  The search for one spectrum follows the
 * step order of Supplementary Algorithm 3 -- precursor filter, shared-peak
 * filter over every peak, score every filtered candidate, keep a heap of the
 * best -- and the statistics follow Supplementary Algorithm 4 and the
 * Superstep 4 text (histogram -> Savitzky-Golay -> tail fit -> expect value).
 * It does NOT use a fragment-ion index: every window candidate's b/y ions are
 * generated directly and compared against the spectrum's peaks.
 *
 * Readings of points the paper leaves open (each stated where it is used):
 *   masses are int64 micro-Dalton (uDa); peaks/precursor are converted once by
 *   llround(x * 1e6); fragment bins are 0.01 Da wide, rounded half up;
 *   fragment charges c = 1..max(1, z-1); shared pairs count (peak, c, ion)
 *   triples with |bin difference| <= T; hyperscore is the X!Tandem form
 *   log10(n_b! * n_y! * S) written as sums of log10; intensities become integer
 *   q in [1, 100] relative to the spectrum's most intense peak; histogram bins
 *   are 0.1 wide in hyperscore (512 int32 bins = 2048 bytes); the survival fit
 *   runs from the smoothed histogram's mode to the bin below the top hit; the
 *   expect value is N * 10^(w * H1 + b) with N the number of scored candidates.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* Monoisotopic residue masses in uDa (standard values; indexed by letter). */
static const int64_t kResidue[26] = {
    /* A */ 71037114, /* B */ -1, /* C */ 103009185, /* D */ 115026943,
    /* E */ 129042593, /* F */ 147068414, /* G */ 57021464, /* H */ 137058912,
    /* I */ 113084064, /* J */ -1, /* K */ 128094963, /* L */ 113084064,
    /* M */ 131040485, /* N */ 114042927, /* O */ -1, /* P */ 97052764,
    /* Q */ 128058578, /* R */ 156101111, /* S */ 87032028, /* T */ 101047679,
    /* U */ -1, /* V */ 99068414, /* W */ 186079313, /* X */ -1,
    /* Y */ 163063329, /* Z */ -1,
};
static const int64_t kWater = 18010565;
static const int64_t kProton = 1007276;
/* Other ion series (the Mod Distance text says the method generalises to a, c,
 * x and z ions): a = b - CO, c = b + NH3, x = y + CO - H2, z = y - NH3.  Masses
 * from the elements: CO 27.994915, NH3 17.026549, H2 2.015650 Da. */
static const int64_t kCO = 27994915;
static const int64_t kNH3 = 17026549;
static const int64_t kH2 = 2015650;
static const int64_t kBinWidth = 10000;   /* 0.01 Da */

/* ------------------------------------------------------------------------ */
/* Database generation (Superstep 1; Supplementary Algorithm 1).             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t  mass;
    uint32_t prot, start, len, pad;
    uint64_t mask;
} peptide;

struct orc_db {
    char*     seq;
    uint64_t* off;
    uint64_t  n_prot;
    uint32_t  n_mods;
    uint32_t  mod_res_mask[ORC_MAX_MODS];
    int32_t   mod_nterm[ORC_MAX_MODS];
    int64_t   mod_delta[ORC_MAX_MODS];
    peptide*  pep;
    uint64_t  n_pep, cap_pep;
};

static int64_t residue_mass(char c) {
    if (c < 'A' || c > 'Z') return -1;
    return kResidue[c - 'A'];
}

/* Trypsin (Experimental Setup): cut after K or R unless the next residue is P. */
static int cleaves_after(const char* s, uint64_t n, uint64_t i) {
    if (s[i] != 'K' && s[i] != 'R') return 0;
    return (i + 1 >= n) || s[i + 1] != 'P';
}

/* Modification sites of a peptide, in mask-bit order: the protein N-terminus
 * first (only when the peptide starts the protein), then residues by position.
 * Reading: each site carries at most one modification. */
typedef struct { uint32_t pos; uint32_t mod; } site;

static uint32_t peptide_sites(const orc_db* db, const char* p, uint32_t len, int at_nterm, site* out) {
    uint32_t n = 0;
    if (at_nterm)
        for (uint32_t m = 0; m < db->n_mods; ++m)
            if (db->mod_nterm[m]) { out[n].pos = 0; out[n].mod = m; ++n; break; }
    for (uint32_t j = 0; j < len; ++j)
        for (uint32_t m = 0; m < db->n_mods; ++m)
            if (!db->mod_nterm[m] && (db->mod_res_mask[m] >> (p[j] - 'A') & 1u)) {
                out[n].pos = j; out[n].mod = m; ++n; break;
            }
    return n;
}

/* Where enumerated entries go: counted only (out == NULL), or written at out[n]. */
typedef struct { peptide* out; uint64_t n; } sink;

static void push_peptide(sink* k, peptide v) {
    if (k->out) k->out[k->n] = v;
    ++k->n;
}

/* All site subsets of size <= max_mods (the 2^m variants of a sequence). */
static void enumerate_variants(const orc_db* db, sink* k, const site* sites, uint32_t n_sites, uint32_t next,
                               uint32_t left, uint64_t mask, int64_t mass, peptide base) {
    base.mask = mask;
    base.mass = mass;
    push_peptide(k, base);
    if (left == 0) return;
    for (uint32_t i = next; i < n_sites; ++i)
        enumerate_variants(db, k, sites, n_sites, i + 1, left - 1, mask | (1ull << i),
                           mass + db->mod_delta[sites[i].mod], base);
}

static int peptide_key_cmp(const void* a, const void* b) {
    const peptide* x = (const peptide*)a;
    const peptide* y = (const peptide*)b;
    if (x->mass != y->mass) return x->mass < y->mass ? -1 : 1;
    if (x->prot != y->prot) return x->prot < y->prot ? -1 : 1;
    if (x->start != y->start) return x->start < y->start ? -1 : 1;
    if (x->len != y->len) return x->len < y->len ? -1 : 1;
    if (x->mask != y->mask) return x->mask < y->mask ? -1 : 1;
    return 0;
}

/* Every peptide of proteins [p0, p1) and its modified forms, into k. */
static void digest_range(const orc_db* db, uint64_t p0, uint64_t p1, uint32_t missed, uint32_t min_len,
                         uint32_t max_len, uint32_t max_mods, sink* k) {
    site sites[64];
    for (uint64_t p = p0; p < p1; ++p) {
        const char* s = db->seq + db->off[p];
        uint64_t n = db->off[p + 1] - db->off[p];
        for (uint64_t a = 0; a < n; ++a) {
            if (a != 0 && !cleaves_after(s, n, a - 1)) continue;   /* a must start a fragment */
            uint32_t missed_here = 0;
            int64_t mass = kWater;
            for (uint64_t e = a + 1; e <= n; ++e) {
                uint64_t len = e - a;
                if (len > max_len) break;
                mass += residue_mass(s[e - 1]);
                int is_end = (e == n) || cleaves_after(s, n, e - 1);
                if (!is_end) continue;
                if (len >= min_len) {
                    peptide base;
                    memset(&base, 0, sizeof base);
                    base.prot = (uint32_t)p;
                    base.start = (uint32_t)a;
                    base.len = (uint32_t)len;
                    uint32_t ns = peptide_sites(db, s + a, (uint32_t)len, a == 0, sites);
                    enumerate_variants(db, k, sites, ns, 0, max_mods, 0, mass, base);
                }
                if (e < n && ++missed_here > missed) break;
            }
        }
    }
}

/* The database is built with several threads, which changes nothing in what it
 * holds: each thread digests a range of proteins (a counting pass sizes the
 * array, a second pass writes each range at its offset), and the entries are
 * sorted by the key above -- which is unique per entry, so the order is the
 * same for any correct sort -- in qsort-sorted chunks merged pairwise. */
typedef struct {
    const orc_db* db; uint64_t p0, p1; uint32_t missed, min_len, max_len, max_mods; sink k;
} digest_job;

static void* digest_worker(void* arg) {
    digest_job* J = (digest_job*)arg;
    digest_range(J->db, J->p0, J->p1, J->missed, J->min_len, J->max_len, J->max_mods, &J->k);
    return NULL;
}

typedef struct { peptide* a; uint64_t n; } sort_job;

static void* sort_worker(void* arg) {
    sort_job* J = (sort_job*)arg;
    qsort(J->a, J->n, sizeof(peptide), peptide_key_cmp);
    return NULL;
}

typedef struct { const peptide* x; uint64_t nx; const peptide* y; uint64_t ny; peptide* out; } merge_job;

static void* merge_worker(void* arg) {
    merge_job* J = (merge_job*)arg;
    uint64_t i = 0, j = 0, o = 0;
    while (i < J->nx && j < J->ny) J->out[o++] = peptide_key_cmp(&J->y[j], &J->x[i]) < 0 ? J->y[j++] : J->x[i++];
    while (i < J->nx) J->out[o++] = J->x[i++];
    while (j < J->ny) J->out[o++] = J->y[j++];
    return NULL;
}

/* Sorts db->pep (n entries) by the key with `threads` threads; returns 0, or -1
 * when the merge buffer cannot be allocated. */
static int sort_entries(orc_db* db, int threads) {
    const uint64_t n = db->n_pep;
    if (threads <= 1 || n < (1u << 16)) { qsort(db->pep, n, sizeof(peptide), peptide_key_cmp); return 0; }
    uint64_t* cut = (uint64_t*)malloc(((size_t)threads + 1) * sizeof(uint64_t));
    for (int t = 0; t <= threads; ++t) cut[t] = n * (uint64_t)t / (uint64_t)threads;
    pthread_t* th = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
    sort_job* sj = (sort_job*)calloc((size_t)threads, sizeof(sort_job));
    for (int t = 0; t < threads; ++t) {
        sj[t].a = db->pep + cut[t]; sj[t].n = cut[t + 1] - cut[t];
        pthread_create(&th[t], NULL, sort_worker, &sj[t]);
    }
    for (int t = 0; t < threads; ++t) pthread_join(th[t], NULL);
    peptide* buf = (peptide*)malloc(n * sizeof(peptide));
    if (!buf) { free(cut); free(th); free(sj); return -1; }
    int runs = threads;
    peptide* src = db->pep;
    peptide* dst = buf;
    merge_job* mj = (merge_job*)calloc((size_t)threads, sizeof(merge_job));
    while (runs > 1) {
        int m = 0;
        for (int r = 0; r < runs; r += 2, ++m) {
            mj[m].out = dst + cut[r];
            mj[m].x = src + cut[r]; mj[m].nx = cut[r + 1] - cut[r];
            if (r + 1 < runs) { mj[m].y = src + cut[r + 1]; mj[m].ny = cut[r + 2] - cut[r + 1]; }
            else { mj[m].y = NULL; mj[m].ny = 0; }
            pthread_create(&th[m], NULL, merge_worker, &mj[m]);
        }
        for (int t = 0; t < m; ++t) pthread_join(th[t], NULL);
        int k = 0;
        for (int r = 0; r < runs; r += 2) cut[k++] = cut[r];
        cut[k] = n;
        runs = k;
        peptide* tmp = src; src = dst; dst = tmp;
    }
    if (src != db->pep) { memcpy(db->pep, src, n * sizeof(peptide)); }
    free(buf); free(cut); free(th); free(sj); free(mj);
    return 0;
}

orc_db* orc_db_create(const char* residues, const uint64_t* prot_off, uint64_t n_prot,
                      uint32_t missed, uint32_t min_len, uint32_t max_len,
                      uint32_t n_mods, const uint32_t* mod_res_mask, const int32_t* mod_nterm,
                      const int64_t* mod_delta, uint32_t max_mods, int threads) {
    if (n_mods > ORC_MAX_MODS || min_len < 2 || max_len < min_len || max_len > 62) return NULL;
    uint64_t total = prot_off[n_prot];
    for (uint64_t i = 0; i < total; ++i)
        if (residue_mass(residues[i]) < 0) return NULL;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    orc_db* db = (orc_db*)calloc(1, sizeof(orc_db));
    db->seq = (char*)malloc(total + 1);
    memcpy(db->seq, residues, total);
    db->off = (uint64_t*)malloc((n_prot + 1) * sizeof(uint64_t));
    memcpy(db->off, prot_off, (n_prot + 1) * sizeof(uint64_t));
    db->n_prot = n_prot;
    db->n_mods = n_mods;
    for (uint32_t m = 0; m < n_mods; ++m) {
        db->mod_res_mask[m] = mod_res_mask[m];
        db->mod_nterm[m] = mod_nterm[m];
        db->mod_delta[m] = mod_delta[m];
    }
    /* count, allocate, then write each thread's protein range at its offset */
    digest_job* J = (digest_job*)calloc((size_t)threads, sizeof(digest_job));
    pthread_t* th = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
    for (int pass = 0; pass < 2; ++pass) {
        uint64_t at = 0;
        for (int t = 0; t < threads; ++t) {
            J[t].db = db;
            J[t].p0 = n_prot * (uint64_t)t / (uint64_t)threads;
            J[t].p1 = n_prot * (uint64_t)(t + 1) / (uint64_t)threads;
            J[t].missed = missed; J[t].min_len = min_len; J[t].max_len = max_len; J[t].max_mods = max_mods;
            if (pass == 1) { J[t].k.out = db->pep + at; at += J[t].k.n; }
            J[t].k.n = 0;
            pthread_create(&th[t], NULL, digest_worker, &J[t]);
        }
        for (int t = 0; t < threads; ++t) pthread_join(th[t], NULL);
        if (pass == 0) {
            uint64_t n = 0;
            for (int t = 0; t < threads; ++t) n += J[t].k.n;
            db->pep = (peptide*)malloc((n ? n : 1) * sizeof(peptide));
            db->n_pep = db->cap_pep = n;
            if (!db->pep) { free(J); free(th); orc_db_free(db); return NULL; }
        }
    }
    free(J);
    free(th);
    if (sort_entries(db, threads) != 0) { orc_db_free(db); return NULL; }
    return db;
}

void orc_db_free(orc_db* db) {
    if (!db) return;
    free(db->seq); free(db->off); free(db->pep); free(db);
}

uint64_t orc_db_size(const orc_db* db) { return db->n_pep; }

void orc_db_get(const orc_db* db, uint64_t id, int64_t* mass, uint32_t* prot,
                uint32_t* start, uint32_t* len, uint64_t* mask) {
    const peptide* p = &db->pep[id];
    *mass = p->mass; *prot = p->prot; *start = p->start; *len = p->len; *mask = p->mask;
}

uint32_t orc_db_residue_masses(const orc_db* db, uint64_t id, int64_t* out, uint32_t cap) {
    const peptide* p = &db->pep[id];
    const char* s = db->seq + db->off[p->prot] + p->start;
    if (p->len > cap) return 0;
    for (uint32_t j = 0; j < p->len; ++j) out[j] = residue_mass(s[j]);
    site sites[64];
    uint32_t ns = peptide_sites(db, s, p->len, p->start == 0, sites);
    for (uint32_t i = 0; i < ns; ++i)
        if (p->mask >> i & 1ull) out[sites[i].pos] += db->mod_delta[sites[i].mod];
    return p->len;
}

/* b/y ions only (Superstep 1 footnote), i = 1..n-1.  The worked Mod Distance
 * example (Supplementary Text 3) counts the first b ion and the first y ion,
 * so the series runs b1..b(n-1), y1..y(n-1). */
void orc_ions(const int64_t* r, uint32_t n, int64_t* b_out, int64_t* y_out) {
    int64_t total = 0;
    for (uint32_t j = 0; j < n; ++j) total += r[j];
    int64_t prefix = 0;
    for (uint32_t i = 1; i < n; ++i) {
        prefix += r[i - 1];
        b_out[i - 1] = prefix + kProton;                    /* residues 1..i */
    }
    int64_t suffix = 0;
    for (uint32_t i = 1; i < n; ++i) {
        suffix += r[n - i];
        y_out[i - 1] = suffix + kWater + kProton;           /* residues n-i+1..n */
    }
    (void)total;
}

/* ------------------------------------------------------------------------ */
/* Scoring pieces.                                                            */
/* ------------------------------------------------------------------------ */

/* Hyperscore, cited by the paper (Superstep 3 cost analysis) from X!Tandem:
 * log10(n_b! * n_y! * sum of matched intensities), taken as
 * (sum_{k=2..n_b} log10 k + sum_{k=2..n_y} log10 k) + log10(S), each sum
 * accumulated left to right. */
static double log10_factorial(uint32_t n) {
    double acc = 0.0;
    for (uint32_t k = 2; k <= n; ++k) acc += log10((double)k);
    return acc;
}

#define LF_CAP 4096
static double g_lf[LF_CAP + 1];
static pthread_once_t g_lf_once = PTHREAD_ONCE_INIT;
static void lf_init(void) {
    double acc = 0.0;
    g_lf[0] = 0.0; g_lf[1] = 0.0;
    for (uint32_t k = 2; k <= LF_CAP; ++k) { acc += log10((double)k); g_lf[k] = acc; }
}
static double lf(uint32_t n) {
    pthread_once(&g_lf_once, lf_init);
    return n <= LF_CAP ? g_lf[n] : log10_factorial(n);
}

double orc_hyperscore(uint32_t n_b, uint32_t n_y, uint32_t sum_q) {
    double h = lf(n_b) + lf(n_y);
    return h + log10((double)sum_q);
}

static int hist_bin(double h) {
    double t = floor(10.0 * h);
    if (t >= ORC_HIST_BINS - 1) return ORC_HIST_BINS - 1;
    return (int)t;
}

/* Savitzky-Golay smoothing (Superstep 4): 5-point quadratic window
 * (-3, 12, 17, 12, -3) / 35, zero outside the histogram, negatives set to 0. */
void orc_sg_smooth(const int32_t* h, double* out) {
    static const double c[5] = {-3.0, 12.0, 17.0, 12.0, -3.0};
    for (int j = 0; j < ORC_HIST_BINS; ++j) {
        double acc = 0.0;
        for (int t = -2; t <= 2; ++t) {
            int i = j + t;
            if (i >= 0 && i < ORC_HIST_BINS) acc += c[t + 2] * (double)h[i];
        }
        acc = acc / 35.0;
        out[j] = acc < 0.0 ? 0.0 : acc;
    }
}

/* Linear tail fit (Superstep 4, after Fenyo & Beavis 2003) and expect value
 * (Supplementary Algorithm 4).  Survival S_j = sum_{i>=j} hs[i] / sum hs;
 * fit log10 S_j = w * (0.1 j) + b by least squares over j from the mode of hs
 * (lowest index on ties) to bin(H1) - 1, skipping S_j = 0.  The printed
 * ev = (w * g_max + b) * size is read in the log domain: ev = N * 10^(w*H1 + b).
 * Returns the status code (0 ok, 1 nothing scored, 2 < 3 points, 3 w >= 0). */
int orc_evalue(const int32_t* hist, double top_h, uint64_t n_scored,
               double* evalue, double* slope, double* intercept, int32_t* n_points) {
    *evalue = NAN; *slope = NAN; *intercept = NAN; *n_points = 0;
    if (n_scored == 0) return 1;
    double hs[ORC_HIST_BINS];
    orc_sg_smooth(hist, hs);
    double total = 0.0;
    for (int j = 0; j < ORC_HIST_BINS; ++j) total += hs[j];
    int mode = 0;
    for (int j = 1; j < ORC_HIST_BINS; ++j) if (hs[j] > hs[mode]) mode = j;
    int last = hist_bin(top_h) - 1;
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    int n = 0;
    if (total > 0.0) {
        for (int j = mode; j <= last; ++j) {
            double tail = 0.0;
            for (int i = j; i < ORC_HIST_BINS; ++i) tail += hs[i];
            double surv = tail / total;
            if (!(surv > 0.0)) continue;
            double x = 0.1 * (double)j;
            double y = log10(surv);
            sx += x; sy += y; sxx += x * x; sxy += x * y; ++n;
        }
    }
    *n_points = n;
    if (n < 3) return 2;
    double w = ((double)n * sxy - sx * sy) / ((double)n * sxx - sx * sx);
    double b = (sy - w * sx) / (double)n;
    *slope = w; *intercept = b;
    if (!(w < 0.0)) return 3;
    *evalue = (double)n_scored * pow(10.0, w * top_h + b);
    return 0;
}

/* The window of ORC_SAMPLE_BINS bins the Sampling section keeps (see
 * orc_sampled): its first bin, or -1 when no bin holds a count. */
static int sample_window(const int32_t* hist) {
    /* the three most intense samples (largest counts; ties go to the lower bin) */
    int top[3];
    int t = 0;
    for (int r = 0; r < 3; ++r) {
        int best = -1;
        for (int j = 0; j < ORC_HIST_BINS; ++j) {
            if (hist[j] <= 0) continue;
            int used = 0;
            for (int u = 0; u < t; ++u) used |= top[u] == j;
            if (used) continue;
            if (best < 0 || hist[j] > hist[best]) best = j;
        }
        if (best < 0) break;
        top[t++] = best;
    }
    if (t == 0) return -1;
    int sum = 0;
    for (int u = 0; u < t; ++u) sum += top[u];
    const int mean = sum / t;                 /* average location, floored */
    int first = 0;
    while (hist[first] <= 0) ++first;
    /* the window reaches down to the head's start, but no further than
     * ORC_SAMPLE_HEAD bins below the mean; what does not fit is tail */
    int lo = first > mean - ORC_SAMPLE_HEAD ? first : mean - ORC_SAMPLE_HEAD;
    if (lo > ORC_HIST_BINS - ORC_SAMPLE_BINS) lo = ORC_HIST_BINS - ORC_SAMPLE_BINS;
    return lo;
}

/* log-Weibull (Gumbel) fit (Superstep 4; Supplementary Algorithm 4 names it
 * next to the tail fit) and expect value.  Reading: the fit sees the samples
 * the Sampling section keeps, the histogram restricted to the ORC_SAMPLE_BINS-bin
 * window of sample_window (zero outside), whose pruned far tail the fitted
 * distribution stands in for; so a partition's 256-byte record and its full
 * histogram give the same fit.  The Gumbel location mu and scale beta come
 * from the moments of the smoothed restricted histogram hs, each bin j standing
 * at its centre x_j = 0.1 j + 0.05: mean m = sum hs x / sum hs, variance
 * v = sum hs (x - m)^2 / sum hs, beta = sqrt(6 v) / pi, mu = m - gamma * beta
 * (gamma = Euler-Mascheroni).  ev = N * S(H1) with the Gumbel survival
 * S(h) = 1 - exp(-exp(-(h - mu) / beta)).  Returns 0 ok, 1 nothing scored, 2
 * fewer than 3 bins of hs above zero. */
int orc_evalue_gumbel(const int32_t* hist, double top_h, uint64_t n_scored,
                      double* evalue, double* mu, double* beta, int32_t* n_points) {
    static const double kEulerGamma = 0.57721566490153286061;
    static const double kPi = 3.14159265358979323846;
    *evalue = NAN; *mu = NAN; *beta = NAN; *n_points = 0;
    if (n_scored == 0) return 1;
    int32_t kept[ORC_HIST_BINS];
    const int lo = sample_window(hist);
    for (int j = 0; j < ORC_HIST_BINS; ++j)
        kept[j] = (lo >= 0 && j >= lo && j < lo + ORC_SAMPLE_BINS && hist[j] > 0) ? hist[j] : 0;
    double hs[ORC_HIST_BINS];
    orc_sg_smooth(kept, hs);
    double w = 0.0, wx = 0.0;
    int n = 0;
    for (int j = 0; j < ORC_HIST_BINS; ++j) {
        if (hs[j] > 0.0) ++n;
        w += hs[j];
        wx += hs[j] * (0.1 * (double)j + 0.05);
    }
    *n_points = n;
    if (n < 3) return 2;
    double m = wx / w;
    double v = 0.0;
    for (int j = 0; j < ORC_HIST_BINS; ++j) {
        double d = (0.1 * (double)j + 0.05) - m;
        v += hs[j] * d * d;
    }
    v = v / w;
    double b = sqrt(6.0 * v) / kPi;
    *beta = b;
    *mu = m - kEulerGamma * b;
    *evalue = (double)n_scored * -expm1(-exp(-(top_h - *mu) / b));
    return 0;
}

static int expect_value(int32_t fit, const int32_t* hist, double top_h, uint64_t n_scored, double* ev) {
    double a, b; int32_t npts;
    if (fit == ORC_FIT_GUMBEL) return orc_evalue_gumbel(hist, top_h, n_scored, ev, &a, &b, &npts);
    return orc_evalue(hist, top_h, n_scored, ev, &a, &b, &npts);
}

/* ------------------------------------------------------------------------ */
/* Search (Supplementary Algorithm 3).                                        */
/* ------------------------------------------------------------------------ */

typedef struct { int64_t bin; uint32_t q; } entry;

typedef struct { uint64_t idx; float mz, in; } peak_ref;

/* Top-B order: intensity descending, then m/z ascending, then input order. */
static int peak_rank_cmp(const void* a, const void* b) {
    const peak_ref* x = (const peak_ref*)a;
    const peak_ref* y = (const peak_ref*)b;
    if (x->in != y->in) return x->in > y->in ? -1 : 1;
    if (x->mz != y->mz) return x->mz < y->mz ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

static int entry_cmp(const void* a, const void* b) {
    const entry* x = (const entry*)a;
    const entry* y = (const entry*)b;
    if (x->bin != y->bin) return x->bin < y->bin ? -1 : 1;
    return (x->q > y->q) - (x->q < y->q);
}

static int64_t bin_of(int64_t m) { return (m + kBinWidth / 2) / kBinWidth; }

/* Superstep 2 pre-processing and sub-task R's top-B selection, then the peak
 * list expanded over fragment charges.  Returns the number of entries, or -1
 * on invalid input. */
/* Pre-processing (Superstep 2 names normalising and clearing noise; sub-task R
 * keeps the B most intense peaks).  Readings: noise clearing drops the peaks
 * with I < Imax * p / 1000 before the top-B selection (p = noise_permille; the
 * comparison I * 1000 >= Imax * p is exact in fp64); intensities become integer
 * q in [1, 100] relative to the most intense peak, linearly or through the
 * square root: q = round half up of 100 * sqrt(I / Imax), taken as the largest
 * k with (k - 1/2)^2 <= 10^4 * I / Imax so that no square root is rounded. */
static int64_t prepare_spectrum(const float* mz, const float* in, uint64_t np, int z,
                                const orc_params* P, entry* out) {
    if (z < 1 || z > 8) return -1;
    peak_ref* r = (peak_ref*)malloc((np ? np : 1) * sizeof(peak_ref));
    float imax = 0.0f;
    for (uint64_t i = 0; i < np; ++i) {
        if (!(mz[i] > 0.0f) || !isfinite(mz[i]) || !(in[i] >= 0.0f) || !isfinite(in[i])) {
            free(r); return -1;
        }
        if (in[i] > imax) imax = in[i];
    }
    uint64_t alive = 0;
    for (uint64_t i = 0; i < np; ++i) {
        if ((double)in[i] * 1000.0 < (double)imax * (double)P->noise_permille) continue;   /* noise */
        r[alive].idx = i; r[alive].mz = mz[i]; r[alive].in = in[i];
        ++alive;
    }
    qsort(r, alive, sizeof(peak_ref), peak_rank_cmp);
    uint64_t keep = alive < P->top_peaks ? alive : P->top_peaks;
    int cmax = z - 1 > 1 ? z - 1 : 1;
    int64_t n = 0;
    for (uint64_t k = 0; k < keep; ++k) {
        /* normalise to the most intense peak: integer q in [1, 100] */
        uint32_t q = 1;
        if (imax > 0.0f && P->intensity == ORC_INTENSITY_SQRT) {
            double t = (double)r[k].in / (double)imax;
            t = t * 10000.0;
            q = 1;
            for (uint32_t c = 100; c >= 1; --c) {
                if (((double)c - 0.5) * ((double)c - 0.5) <= t) { q = c; break; }
            }
        } else if (imax > 0.0f) {
            double t = (double)r[k].in / (double)imax;
            t = t * 100.0;
            t = t + 0.5;
            t = floor(t);
            q = t < 1.0 ? 1u : (t > 100.0 ? 100u : (uint32_t)t);
        }
        int64_t mz_uda = llround((double)r[k].mz * 1e6);
        for (int c = 1; c <= cmax; ++c) {
            int64_t m1 = (int64_t)c * mz_uda - (int64_t)(c - 1) * kProton;  /* singly charged */
            if (m1 < 0) continue;
            out[n].bin = bin_of(m1);
            out[n].q = q;
            ++n;
        }
    }
    free(r);
    qsort(out, (size_t)n, sizeof(entry), entry_cmp);
    return n;
}

/* Number of entries with |bin - x| <= T, and the sum of their q. */
static void match_ion(const entry* e, int64_t n, int64_t x, int64_t T, uint32_t* cnt, uint32_t* qs) {
    int64_t lo = 0, hi = n;                 /* first entry with bin >= x - T */
    while (lo < hi) { int64_t mid = (lo + hi) / 2; if (e[mid].bin < x - T) lo = mid + 1; else hi = mid; }
    for (int64_t i = lo; i < n && e[i].bin <= x + T; ++i) { *cnt += 1; *qs += e[i].q; }
}

typedef struct {
    uint32_t id, n_b, n_y, s;
    double h;
} scored;

static int better(double ha, uint32_t ida, double hb, uint32_t idb) {
    return ha > hb || (ha == hb && ida < idb);
}

typedef struct {
    const orc_db* db;
    const orc_params* prm;
    /* one spectrum */
    const float* mz; const float* in; uint64_t np; double prec; int z;
    /* outputs */
    orc_hit* hits; orc_stat* stat; int32_t* hist;
    /* optional dump of the scored set */
    uint32_t* d_id; uint16_t* d_nb; uint16_t* d_ny; uint32_t* d_s; uint64_t d_cap; int64_t d_n;
} job;

static int search_one(job* J) {
    const orc_db* db = J->db;
    const orc_params* P = J->prm;
    uint32_t k = P->top_k;
    int32_t local_hist[ORC_HIST_BINS];
    memset(local_hist, 0, sizeof local_hist);
    for (uint32_t i = 0; i < k; ++i) {
        J->hits[i].id = UINT32_MAX; J->hits[i].n_b = 0; J->hits[i].n_y = 0;
        J->hits[i].sum_q = 0; J->hits[i].pad = 0; J->hits[i].hyperscore = -INFINITY;
    }
    memset(J->stat, 0, sizeof *J->stat);

    entry* ent = (entry*)malloc((J->np * 8 + 1) * sizeof(entry));
    int64_t ne = prepare_spectrum(J->mz, J->in, J->np, J->z, P, ent);
    if (ne < 0 || !isfinite(J->prec) || J->prec <= 0.0) { free(ent); return -1; }

    /* filter_1: precursor mass window, |M_pep - M_q| <= dM, inclusive. */
    int64_t mq = (int64_t)J->z * (llround(J->prec * 1e6) - kProton);
    if (mq < 0) { free(ent); return -1; }
    int64_t dm = P->window_is_ppm ? (mq * P->window) / 1000000 : P->window;
    uint64_t lo = db->n_pep, hi = 0;
    for (uint64_t id = 0; id < db->n_pep; ++id) {
        int64_t d = db->pep[id].mass - mq;
        if (d >= -dm && d <= dm) { if (id < lo) lo = id; hi = id + 1; }
    }
    if (hi == 0) lo = hi = 0;
    J->stat->lo = lo; J->stat->hi = hi; J->stat->n_window = hi - lo;

    /* filter_2 + score: generate each candidate's ions, count shared peaks.
     * Reading for other ion series: matches of N-terminal ions (a, b, c) count
     * in n_b and of C-terminal ions (x, y, z) in n_y, so the hyperscore keeps
     * its two factorials. */
    const uint32_t types = P->ion_types ? P->ion_types : (ORC_ION_B | ORC_ION_Y);
    int64_t res[64], bi[64], yi[64];
    uint64_t n_scored = 0, pairs_total = 0;
    for (uint64_t id = lo; id < hi; ++id) {
        uint32_t n = orc_db_residue_masses(db, id, res, 64);
        orc_ions(res, n, bi, yi);
        uint32_t nb = 0, ny = 0, sq = 0;
        for (uint32_t i = 0; i + 1 < n; ++i) {
            if (types & ORC_ION_A) match_ion(ent, ne, bin_of(bi[i] - kCO), P->frag_tol_bins, &nb, &sq);
            if (types & ORC_ION_B) match_ion(ent, ne, bin_of(bi[i]), P->frag_tol_bins, &nb, &sq);
            if (types & ORC_ION_C) match_ion(ent, ne, bin_of(bi[i] + kNH3), P->frag_tol_bins, &nb, &sq);
            if (types & ORC_ION_X) match_ion(ent, ne, bin_of(yi[i] + kCO - kH2), P->frag_tol_bins, &ny, &sq);
            if (types & ORC_ION_Y) match_ion(ent, ne, bin_of(yi[i]), P->frag_tol_bins, &ny, &sq);
            if (types & ORC_ION_Z) match_ion(ent, ne, bin_of(yi[i] - kNH3), P->frag_tol_bins, &ny, &sq);
        }
        pairs_total += nb + ny;
        if (nb + ny < P->min_shared) continue;        /* shared peaks >= k */
        double h = orc_hyperscore(nb, ny, sq);
        ++n_scored;
        local_hist[hist_bin(h)] += 1;
        if (J->d_id) {
            if ((uint64_t)J->d_n < J->d_cap) {
                J->d_id[J->d_n] = (uint32_t)id; J->d_nb[J->d_n] = (uint16_t)nb;
                J->d_ny[J->d_n] = (uint16_t)ny; J->d_s[J->d_n] = sq;
            }
            ++J->d_n;
        }
        /* heap of the k best, ordered by (hyperscore desc, id asc) */
        if (k && better(h, (uint32_t)id, J->hits[k - 1].hyperscore, J->hits[k - 1].id)) {
            uint32_t pos = k - 1;
            while (pos > 0 && better(h, (uint32_t)id, J->hits[pos - 1].hyperscore, J->hits[pos - 1].id)) {
                J->hits[pos] = J->hits[pos - 1];
                --pos;
            }
            J->hits[pos].id = (uint32_t)id; J->hits[pos].n_b = (uint16_t)nb;
            J->hits[pos].n_y = (uint16_t)ny; J->hits[pos].sum_q = sq; J->hits[pos].pad = 0;
            J->hits[pos].hyperscore = h;
        }
    }
    free(ent);
    J->stat->n_scored = n_scored;
    J->stat->pairs_total = pairs_total;
    if (J->hist) memcpy(J->hist, local_hist, sizeof local_hist);
    double top = n_scored ? J->hits[0].hyperscore : 0.0;     /* k >= 1 is enforced */
    J->stat->status = expect_value(P->fit, local_hist, top, n_scored, &J->stat->evalue);
    return 0;
}

typedef struct {
    const orc_db* db; const orc_params* prm;
    uint64_t n; const uint64_t* off; const float* mz; const float* in;
    const double* prec; const int8_t* z;
    orc_hit* hits; orc_stat* stats; int32_t* hist;
    int tid, nthreads; int err;
} worker;

static void* work_loop(void* arg) {
    worker* W = (worker*)arg;
    for (uint64_t s = (uint64_t)W->tid; s < W->n; s += (uint64_t)W->nthreads) {
        job J;
        memset(&J, 0, sizeof J);
        J.db = W->db; J.prm = W->prm;
        J.mz = W->mz + W->off[s]; J.in = W->in + W->off[s]; J.np = W->off[s + 1] - W->off[s];
        J.prec = W->prec[s]; J.z = W->z[s];
        J.hits = W->hits + s * W->prm->top_k; J.stat = W->stats + s;
        J.hist = W->hist ? W->hist + s * ORC_HIST_BINS : NULL;
        if (search_one(&J) != 0) W->err = 1;
    }
    return NULL;
}

static int params_ok(const orc_params* P) {
    return P->top_k >= 1 && P->top_k <= 64 && P->min_shared >= 1 && P->frag_tol_bins >= 0 &&
           (P->fit == ORC_FIT_TAIL || P->fit == ORC_FIT_GUMBEL) && P->noise_permille <= 1000 &&
           (P->intensity == ORC_INTENSITY_LINEAR || P->intensity == ORC_INTENSITY_SQRT) && P->ion_types < 64u &&
           P->window >= 0 && P->top_peaks >= 1;
}

int orc_search(const orc_db* db, uint64_t n, const uint64_t* peak_off, const float* mz,
               const float* intensity, const double* precursor_mz, const int8_t* charge,
               const orc_params* P, int threads, orc_hit* hits, orc_stat* stats, int32_t* hist) {
    if (!params_ok(P)) return -1;
    if (threads < 1) threads = 1;
    worker* W = (worker*)calloc((size_t)threads, sizeof(worker));
    pthread_t* th = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
    for (int t = 0; t < threads; ++t) {
        W[t].db = db; W[t].prm = P; W[t].n = n; W[t].off = peak_off; W[t].mz = mz;
        W[t].in = intensity; W[t].prec = precursor_mz; W[t].z = charge;
        W[t].hits = hits; W[t].stats = stats; W[t].hist = hist; W[t].tid = t; W[t].nthreads = threads;
        pthread_create(&th[t], NULL, work_loop, &W[t]);
    }
    int err = 0;
    for (int t = 0; t < threads; ++t) { pthread_join(th[t], NULL); err |= W[t].err; }
    free(W); free(th);
    return err ? -1 : 0;
}

int64_t orc_scored(const orc_db* db, const uint64_t* peak_off_2, const float* mz,
                   const float* intensity, double precursor_mz, int8_t charge,
                   const orc_params* P, uint32_t* ids, uint16_t* n_b, uint16_t* n_y,
                   uint32_t* sum_q, uint64_t cap) {
    if (!params_ok(P)) return -1;
    orc_hit* hits = (orc_hit*)calloc(P->top_k, sizeof(orc_hit));
    orc_stat st;
    job J;
    memset(&J, 0, sizeof J);
    J.db = db; J.prm = P;
    J.mz = mz + peak_off_2[0]; J.in = intensity + peak_off_2[0]; J.np = peak_off_2[1] - peak_off_2[0];
    J.prec = precursor_mz; J.z = charge; J.hits = hits; J.stat = &st; J.hist = NULL;
    J.d_id = ids; J.d_nb = n_b; J.d_ny = n_y; J.d_s = sum_q; J.d_cap = cap; J.d_n = 0;
    int rc = search_one(&J);
    free(hits);
    return rc ? -1 : J.d_n;
}

/* ------------------------------------------------------------------------ */
/* Partitions and result assembly (Superstep 1 is_mine; Superstep 4;          */
/* Supplementary Algorithm 4).                                                */
/* ------------------------------------------------------------------------ */

/* The entries a process keeps in a partitioned search.  Reading: the sorted
 * database is scattered round robin (Supplementary Fig. 3 allows round robin or
 * random), so entry r of the whole database is entry r / G of partition r % G
 * and every partition keeps the global sort order. */
orc_db* orc_db_shard(const orc_db* src, uint32_t n_shards, uint32_t shard) {
    if (n_shards == 0 || shard >= n_shards) return NULL;
    orc_db* db = (orc_db*)calloc(1, sizeof(orc_db));
    uint64_t total = src->off[src->n_prot];
    db->seq = (char*)malloc(total + 1);
    memcpy(db->seq, src->seq, total);
    db->off = (uint64_t*)malloc((src->n_prot + 1) * sizeof(uint64_t));
    memcpy(db->off, src->off, (src->n_prot + 1) * sizeof(uint64_t));
    db->n_prot = src->n_prot;
    db->n_mods = src->n_mods;
    memcpy(db->mod_res_mask, src->mod_res_mask, sizeof db->mod_res_mask);
    memcpy(db->mod_nterm, src->mod_nterm, sizeof db->mod_nterm);
    memcpy(db->mod_delta, src->mod_delta, sizeof db->mod_delta);
    const uint64_t n = src->n_pep > shard ? (src->n_pep - shard + n_shards - 1) / n_shards : 0;
    db->pep = (peptide*)malloc((n ? n : 1) * sizeof(peptide));
    if (!db->pep) { orc_db_free(db); return NULL; }
    sink k = {db->pep, 0};
    for (uint64_t r = shard; r < src->n_pep; r += n_shards) push_peptide(&k, src->pep[r]);
    db->n_pep = db->cap_pep = k.n;
    return db;
}

static int hit_order_cmp(const void* a, const void* b) {
    const orc_hit* x = (const orc_hit*)a;
    const orc_hit* y = (const orc_hit*)b;
    if (better(x->hyperscore, x->id, y->hyperscore, y->id)) return -1;
    if (better(y->hyperscore, y->id, x->hyperscore, x->id)) return 1;
    return 0;
}

/* Assemble the partial results of G partitions into complete ones, per
 * spectrum, in the order of Supplementary Algorithm 4:
 *   1. the null distribution is the bin-wise sum of the partial histograms
 *      (the "addition" of Superstep 4; the partial histograms here are not
 *      sampled, so they share bin 0 and no shift is needed);
 *   2. every partial top hit, with its id turned back into the global id
 *      (local * G + g), goes into one list ordered by (hyperscore desc,
 *      id asc), of which the first k are kept (the max-heap);
 *   3. the fit and expect value (orc_evalue or orc_evalue_gumbel) run on the assembled histogram
 *      with the best hit's hyperscore and N = the summed scored counts.
 * Window sizes and shared-pair totals add; the window id range is recovered
 * from the partitions' ranges.  Inputs are laid out [G][n][...]. */
int orc_assemble(uint32_t n_shards, uint64_t n, uint32_t top_k, int32_t fit, const orc_hit* part_hits,
                 const orc_stat* part_stats, const int32_t* part_hist, orc_hit* hits,
                 orc_stat* stats, int32_t* hist) {
    if (n_shards == 0 || top_k < 1 || top_k > 64 || (fit != ORC_FIT_TAIL && fit != ORC_FIT_GUMBEL)) return -1;
    const uint64_t G = n_shards;
    orc_hit* pool = (orc_hit*)malloc((size_t)G * top_k * sizeof(orc_hit));
    int32_t dist[ORC_HIST_BINS];
    for (uint64_t s = 0; s < n; ++s) {
        memset(dist, 0, sizeof dist);
        orc_stat st;
        memset(&st, 0, sizeof st);
        uint64_t lo = UINT64_MAX, hi = 0;
        uint64_t m = 0;
        for (uint64_t g = 0; g < G; ++g) {
            const orc_stat* ps = part_stats + g * n + s;
            st.n_window += ps->n_window;
            st.n_scored += ps->n_scored;
            st.pairs_total += ps->pairs_total;
            if (ps->hi > ps->lo) {
                uint64_t a = ps->lo * G + g, b = (ps->hi - 1) * G + g + 1;
                if (a < lo) lo = a;
                if (b > hi) hi = b;
            }
            for (int j = 0; j < ORC_HIST_BINS; ++j) dist[j] += part_hist[(g * n + s) * ORC_HIST_BINS + j];
            const orc_hit* ph = part_hits + (g * n + s) * top_k;
            for (uint32_t i = 0; i < top_k; ++i) {
                if (ph[i].id == UINT32_MAX) continue;
                pool[m] = ph[i];
                pool[m].id = (uint32_t)((uint64_t)ph[i].id * G + g);
                ++m;
            }
        }
        if (hi == 0) lo = 0;
        st.lo = lo; st.hi = hi;
        qsort(pool, (size_t)m, sizeof(orc_hit), hit_order_cmp);
        orc_hit* out = hits + s * top_k;
        for (uint32_t i = 0; i < top_k; ++i) {
            if (i < m) { out[i] = pool[i]; continue; }
            out[i].id = UINT32_MAX; out[i].n_b = 0; out[i].n_y = 0;
            out[i].sum_q = 0; out[i].pad = 0; out[i].hyperscore = -INFINITY;
        }
        double top = st.n_scored ? out[0].hyperscore : 0.0;
        st.status = expect_value(fit, dist, top, st.n_scored, &st.evalue);
        stats[s] = st;
        if (hist) memcpy(hist + s * ORC_HIST_BINS, dist, sizeof dist);
    }
    free(pool);
    return 0;
}

/* Sampling section and its figure: locate the mean of the score distribution
 * from its three most intense samples, then keep ORC_SAMPLE_BINS samples
 * around it, giving up the tail before the head. */
void orc_sample(const int32_t* hist, uint64_t n_scored, orc_sampled* out) {
    memset(out, 0, sizeof *out);
    out->n_scored = n_scored;
    const int lo = sample_window(hist);
    if (lo < 0) return;                       /* empty distribution: nothing to keep */
    out->lo = (uint16_t)lo;
    for (int j = 0; j < ORC_HIST_BINS; ++j) {
        const int32_t v = hist[j] > 0 ? hist[j] : 0;
        if (j >= lo && j < lo + ORC_SAMPLE_BINS) {
            if (v > 65535) out->flags |= 1;
            out->count[j - lo] = (uint16_t)(v > 65535 ? 65535 : v);
        } else if (v > 0) {
            out->flags |= 2;
        }
    }
}

void orc_unsample(const orc_sampled* in, int32_t* hist) {
    memset(hist, 0, ORC_HIST_BINS * sizeof(int32_t));
    if (in->lo > ORC_HIST_BINS - ORC_SAMPLE_BINS) return;   /* not a record orc_sample writes */
    for (int i = 0; i < ORC_SAMPLE_BINS; ++i) hist[in->lo + i] = in->count[i];
}

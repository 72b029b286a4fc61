// state.h -- host-side objects behind the opaque ABI handles.
#pragma once
#include <string>
#include <vector>

#include "internal.h"

namespace ps {

// Record a thread-local error message for ps_last_error(); returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// PS_OK when a gfx950-class device is usable, else PS_EDEVICE (message set).
int require_device();
unsigned worker_threads();
int64_t residue_uda(char c);

// Trypsin: cut after K or R unless the next residue is P.
inline bool is_cut(const char* s, uint64_t n, uint64_t i) {
    if (s[i] != 'K' && s[i] != 'R') return false;
    return i + 1 >= n || s[i + 1] != 'P';
}

void score_tables(std::vector<double>& lf, std::vector<double>& ls);

}  // namespace ps

struct ps_index {
    struct Mod {
        uint32_t res_mask;
        bool nterm;
        int64_t delta;
        std::string residues;
    };
    uint32_t missed = 0, min_len = 0, max_len = 0, max_mods = 0;
    uint32_t merge_tol = 0;      // lists of bin b hold the postings of bins b-T..b+T
    uint32_t n_shards = 1, shard = 0;   // this index holds whole-database ranks r % n_shards == shard
    uint32_t ion_types = PS_ION_B | PS_ION_Y;
    std::vector<Mod> mods;
    std::vector<char> seq;
    std::vector<uint64_t> prot_off;
    // entries sorted by (mass, protein, start, length, mask); id = position (in the partition)
    std::vector<int64_t> mass;
    std::vector<uint32_t> prot, start;
    std::vector<uint8_t> len;
    std::vector<uint64_t> mask;
    // CSR fragment-ion index (host form: lists back to back; on the device each
    // list is padded to whole 16-byte quads)
    uint64_t n_bins = 0;
    std::vector<uint64_t> bin_off;
    std::vector<uint32_t> post;
    uint32_t max_len_seen = 0;
    int64_t min_residue = 0;
    // tile directory: dir[bin * dir_stride + k] = position inside bin's list of its first posting
    // with id >= k << dir_shift
    uint32_t dir_shift = 12;
    uint64_t dir_nblk = 0;       // blocks: entries 0..dir_nblk are meaningful
    uint64_t dir_stride = 0;     // row length, dir_nblk + 1 rounded up to a multiple of 4
    std::vector<uint32_t> dir;
    ps_schedule sched{};
    // device copy
    bool on_device = false;
    ps::DevIndex dev{};
    // entries in the index (the host vectors above hold them unless the index was built on the device)
    uint64_t n_entries = 0;
    // built on the device: postings, directory and the entry table exist only there
    bool device_built = false;
    const uint32_t* dev_prot = nullptr;
    const uint32_t* dev_start = nullptr;
    const uint8_t* dev_len = nullptr;
    const uint64_t* dev_mask = nullptr;
    uint64_t dev_n_post = 0, dev_dir_entries = 0;
    uint64_t dev_n_quads = 0;    // padded postings on the device / 4
    // dense maps (lists holding a large share of the ids), built on the device
    uint32_t n_dense = 0;
    uint32_t dense_bin[ps::kMaxDense] = {};
    bool dense_on = true;        // searches read them (ps_index_set_dense)
};

namespace ps {
int index_prepare(const ps_db_params* params, const char* residues, const uint64_t* prot_off, uint64_t n_proteins,
                  ps_index** out);
int index_build_host(ps_index* ix);

inline uint64_t n_postings(const ps_index* ix) { return ix->device_built ? ix->dev_n_post : ix->post.size(); }
inline uint64_t dir_entries(const ps_index* ix) { return ix->device_built ? ix->dev_dir_entries : ix->dir.size(); }
// Quads of the device postings: every bin's list padded to a multiple of four.
uint64_t padded_quads(const ps_index* ix);

// Device layout of an index block: [mass][bin_q][post][lf][ls][dir], each 256-byte aligned;
// n_quads is the padded postings / 4.
struct DevLayout {
    uint64_t mass, bin, post, lf, ls, dir;
    uint64_t prot, start, mask, len;   // the entry table, kept on the device by a device build (else empty)
    uint64_t dense, dense_stride;      // dense_cap maps of dense_stride bytes
    uint64_t dense_flags;              // u32 [kMaxDense] flags of the candidate maps, then
                                       // u32 [kMaxDense] table of the maps in use (DevIndex::dense_tab)
    uint32_t dense_cap;
    uint64_t total;
};
DevLayout index_layout(uint64_t n_pep, uint64_t n_bins, uint64_t n_quads, uint64_t n_dir, bool entries,
                       uint32_t dense_cap);
// Lists that qualify as dense (at least a quarter of the ids), longest first,
// at most kMaxDense, from the host bin offsets.
std::vector<uint32_t> dense_candidates(const ps_index* ix);
// Build the dense maps of the candidate lists into the index block (after
// bind_device_index) and enable them; a list whose postings repeat an
// (id, terminus) pair keeps no map.  Synchronizes `st`.
int build_dense_maps(ps_index* ix, char* base, const DevLayout& lay, hipStream_t st);
// Point the kernels' view at the maps in use (none while searches are told not to read them).
void bind_dense(ps_index* ix);
// Point ix->dev at an index block laid out by `lay` and mark the index on the device.
void bind_device_index(ps_index* ix, char* base, const DevLayout& lay);
// Modification lookup: which mod (if any) sits on each residue letter; the N-terminal mod.
struct ModTable {
    int res_mod[26];
    int nterm_mod;
};
ModTable mod_table(const ps_index* ix);
int64_t lightest_residue(const ps_index* ix, const ModTable& mt);
// Directory grain for n_pep ids over n_bins bins (4096 ids unless the directory would pass 16 GiB).
uint32_t directory_shift(uint64_t n_bins, uint64_t n_pep);
}

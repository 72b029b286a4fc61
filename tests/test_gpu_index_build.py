"""The fragment-ion index built on the GPU (Superstep 1; needs an MI355X).

ps_index_build_device must give the host build's index bit for bit: every
entry (mass, protein, start, length, site mask), the CSR bin offsets and
postings, and the tile directory, for classic and merged lists, with
modifications (N-terminal ones included), for database partitions and for
degenerate databases.  The host build is itself pinned to the oracle
(test_capi_host.py); searches on the two indexes must agree bit for bit.
"""
import numpy as np
import pytest

from paper_2102_02286_amd import capi, engine, synth

pytestmark = pytest.mark.gpu

ALL_MODS = [synth.OXIDATION, synth.PHOSPHO, synth.ACETYL_NTERM, synth.DEAMIDATION]


def _say(msg):
    print(msg, flush=True)


def _both(prot, missed, min_len, max_len, mods, max_mods, chunk_pairs=0, **kw):
    m = engine.mods_from_synth(mods)
    host = engine.HostIndex(prot.residues, prot.offsets, missed, min_len, max_len, m, max_mods, **kw)
    dev = engine.HostIndex.build_on_device(prot.residues, prot.offsets, missed, min_len, max_len, m, max_mods,
                                           chunk_pairs=chunk_pairs, **kw)
    return host, dev


def _assert_same_index(host, dev):
    assert host.shape() == dev.shape()
    assert host.entries().tobytes() == dev.entries().tobytes()
    oh, ph = host.host_arrays()
    od, pd = dev.host_arrays()
    assert np.array_equal(oh, od), "bin offsets differ"
    assert np.array_equal(ph, pd), "postings differ"
    assert host.directory() == dev.directory()
    assert np.array_equal(host.directory_array(), dev.directory_array()), "tile directories differ"
    assert host.schedule().tile == dev.schedule().tile
    # dense maps: the lists of at least n_pep / 4 postings (longest first, at
    # most eight) without a repeated posting
    L = np.diff(oh.astype(np.int64))
    n_pep = len(host)
    order = np.lexsort((np.arange(L.size), -L))
    cand = [int(b) for b in order[:64] if n_pep and L[b] * 4 >= n_pep][:capi.PS_MAX_DENSE]
    want = [b for b in cand if np.unique(ph[oh[b]:oh[b + 1]]).size == L[b]]
    assert dev.dense()[0].tolist() == want
    # the device-built index keeps its entry table on the device: single entries
    # and peptide strings read back from it equal the host build's
    n = len(host)
    for i in sorted({0, n // 3, n // 2, n - 1} if n else set()):
        assert host.peptide(i) == dev.peptide(i)
        assert host.entry(i) == dev.entry(i)


@pytest.mark.parametrize("mods,max_mods,T,chunk", [([], 0, 0, 0), ([synth.OXIDATION], 2, 1, 0), (ALL_MODS, 3, 2, 0),
                                                   (ALL_MODS, 2, 1, 1 << 22), ([synth.OXIDATION], 2, 0, 1000)])
def test_device_build_equals_host_build(mods, max_mods, T, chunk):
    """chunk > 0 forces the chunked counting sort (many chunks; 1000 pairs is
    raised to one peptide's worth)."""
    prot = synth.make_proteome(300 if chunk != 1000 else 20, seed=3)
    _say(f"device build: {len(mods)} mods, max {max_mods}, merge {T}, chunk {chunk}")
    host, dev = _both(prot, 2, 6, 40, mods, max_mods, chunk_pairs=chunk, merge_tol=T)
    assert len(host) > (10000 if chunk != 1000 else 500)
    _assert_same_index(host, dev)


@pytest.mark.parametrize("types,T", [(63, 1), (4 | 32, 0), (1 | 2 | 16, 2)])
def test_device_build_other_ion_series(types, T):
    prot = synth.make_proteome(150, seed=13)
    _say(f"device build: ion series {types}, merge {T}")
    host, dev = _both(prot, 2, 6, 40, [synth.OXIDATION, synth.ACETYL_NTERM], 2, merge_tol=T, ion_types=types)
    _assert_same_index(host, dev)


@pytest.mark.parametrize("G", [2, 3])
def test_device_build_partitions(G):
    prot = synth.make_proteome(200, seed=11)
    for g in range(G):
        _say(f"device build: partition {g} of {G}")
        host, dev = _both(prot, 1, 7, 30, [synth.OXIDATION, synth.PHOSPHO], 2, chunk_pairs=1 << 20, merge_tol=1,
                          n_shards=G, shard=g)
        _assert_same_index(host, dev)
        # the partition's postings fit the bound the block was sized for
        assert dev.shape()[1] * 4 <= dev.arena.numel()


def test_device_build_degenerate_databases():
    cases = [
        (b"KKRRKPRPKRKKAAKR", 1, 2, 10),               # cleavage sites everywhere, KP / RP not cut
        (b"MPEPTIDE", 0, 2, 20),                        # one protein, no cleavage site
        (b"AK", 2, 2, 2),                                # the shortest peptide
        (b"ACDEFGHIKLMNPQRSTVWY" * 5, 0, 30, 40),       # no peptide in the length range
    ]
    for seq, missed, lo, hi in cases:
        prot = synth.Proteome(np.frombuffer(seq, np.uint8).copy(), np.array([0, len(seq)], np.uint64))
        _say(f"device build: {seq[:20]!r} missed {missed} length {lo}..{hi}")
        host, dev = _both(prot, missed, lo, hi, [synth.ACETYL_NTERM, synth.OXIDATION], 2)
        _assert_same_index(host, dev)
    # several proteins, some empty
    seqs = [b"", b"MKWVTFISLLR", b"", b"GGGGK", b"MSTYK"]
    off = np.zeros(len(seqs) + 1, np.uint64)
    off[1:] = np.cumsum([len(s) for s in seqs])
    prot = synth.Proteome(np.frombuffer(b"".join(seqs), np.uint8).copy(), off)
    host, dev = _both(prot, 1, 2, 20, ALL_MODS, 3, merge_tol=4)
    _assert_same_index(host, dev)


@pytest.fixture(scope="module")
def small_open_pair():
    w = synth.workload("medium")
    prot = synth.make_proteome(2000, seed=0)
    sp = w.spectra(prot, n=96, seed=7)
    host, dev = _both(prot, w.missed, w.min_len, w.max_len, w.mods, w.max_mods, merge_tol=w.frag_tol_bins)
    return w, sp, host.upload(), dev


@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_searches_on_device_built_index(small_open_pair, schedule):
    w, sp, host, dev = small_open_pair
    _say(f"search on the device-built index, schedule {schedule}")
    _assert_same_index(host, dev)
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=schedule)
    a = engine.search(host, sp, prm)
    b = engine.search(dev, sp, prm)
    assert a.hits.tobytes() == b.hits.tobytes()
    assert a.stats.tobytes() == b.stats.tobytes()
    assert a.hist.tobytes() == b.hist.tobytes()
    assert (a.stats["status"] == 0).sum() > 40


def test_device_build_full_medium_database():
    """The full medium database (3.49M entries, 467M merged postings, 1.9 GB
    directory): every array equal to the host build."""
    w = synth.workload("medium")
    prot = w.proteome()
    _say("device build: full medium database")
    host, dev = _both(prot, w.missed, w.min_len, w.max_len, w.mods, w.max_mods, merge_tol=w.frag_tol_bins)
    assert len(dev) == 3486494
    _assert_same_index(host, dev)


@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_device_built_index_search_matches_oracle(schedule):
    """A search on the index built on the GPU compared with the oracle
    directly (not through the host build): the oracle digests and scores every
    window candidate itself.  Merged lists, two modification types, the
    chunked counting sort forced by a small chunk."""
    import oracle
    from tests.test_gpu_parity import assert_parity
    w = synth.workload("medium")
    prot = synth.make_proteome(1500, seed=21)
    mods = [synth.OXIDATION, synth.PHOSPHO]
    sp = w.spectra(prot, n=80, seed=17)
    _say(f"device-built index vs the oracle, schedule {schedule}")
    dev = engine.HostIndex.build_on_device(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                                           engine.mods_from_synth(mods), 2, merge_tol=w.frag_tol_bins,
                                           chunk_pairs=1 << 22)
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, oracle.mods_from_synth(mods), 2)
    assert len(db) == len(dev)
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=schedule)
    res = engine.search(dev, sp, prm)
    oh, ost, og = db.search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
    assert_parity(res, oh, ost, og)
    assert res.postings == int(ost["pairs_total"].sum())
    assert (ost["status"] == 0).sum() > 30

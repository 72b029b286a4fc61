"""Dense lists (needs an MI355X).

Lists holding at least a quarter of the ids (in a tryptic database the y1
ions of K and R) also get a two-bit-per-id map.  A probe on such a list may
skip the stream: the candidate filter then admits ids that could still reach
min_shared with the most the map probes can add, and each admitted id reads
its bits from the maps before the exact test.  Which lists get a map is
checked against the host arrays, and every search must give the
postings-only search's results bit for bit and the oracle's, for closed and
open windows (item edges inside tiles), classic and merged lists, both
schedules, more map probes than an item keeps, and 64-bit counters.
"""
import numpy as np
import pytest

import oracle
from paper_2102_02286_amd import capi, engine, synth

pytestmark = pytest.mark.gpu

Y1_K, Y1_R = 14711, 17512          # y1 of K (147.1128) and R (175.1190) in 0.01-Da bins


def _say(msg):
    print(msg, flush=True)


def _expected_dense(ix):
    """Lists of at least n_pep / 4 postings, longest first (ties by bin), at
    most eight, without a repeated (id, terminus) posting."""
    off, post = ix.host_arrays()
    n = len(ix)
    L = np.diff(off.astype(np.int64))
    order = np.lexsort((np.arange(L.size), -L))
    cand = [int(b) for b in order[:64] if L[b] * 4 >= n][:capi.PS_MAX_DENSE]
    keep = [b for b in cand if np.unique(post[off[b]:off[b + 1]]).size == L[b]]
    return np.array(keep, np.uint32)


def _same(a, b):
    assert a.hits.tobytes() == b.hits.tobytes()
    assert a.stats.tobytes() == b.stats.tobytes()
    assert a.hist.tobytes() == b.hist.tobytes()


def _on_off(ix, sp, prm):
    ix.set_dense(False)
    try:
        r_off = engine.search(ix, sp, prm)
    finally:
        ix.set_dense(True)
    r_on = engine.search(ix, sp, prm)
    return r_on, r_off, r_on, r_off


@pytest.fixture(scope="module")
def open_db():
    w = synth.workload("medium")
    prot = synth.make_proteome(1500, seed=4)
    sp = w.spectra(prot, n=120, seed=6)
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                         oracle.mods_from_synth(w.mods), w.max_mods)
    return w, prot, sp, db


@pytest.mark.parametrize("merge", [0, 1])
def test_dense_maps_are_the_y1_lists(open_db, merge):
    w, prot, sp, db = open_db
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(w.mods), w.max_mods, merge_tol=merge).upload()
    bins, on = ix.dense()
    _say(f"dense bins (merge {merge}): {bins.tolist()}")
    assert on
    assert np.array_equal(bins, _expected_dense(ix))
    want = {Y1_K, Y1_R} if merge == 0 else {Y1_K + d for d in (-1, 0, 1)} | {Y1_R + d for d in (-1, 0, 1)}
    assert want <= set(bins.tolist())


@pytest.mark.parametrize("merge,schedule", [(0, capi.PS_SCHED_PLAIN), (0, capi.PS_SCHED_PERSISTENT),
                                            (1, capi.PS_SCHED_PLAIN), (1, capi.PS_SCHED_PERSISTENT)])
def test_dense_open_search_equals_postings_and_oracle(open_db, merge, schedule):
    w, prot, sp, db = open_db
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(w.mods), w.max_mods, merge_tol=merge).upload()
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=schedule)
    _say(f"dense open search: merge {merge}, schedule {schedule}")
    r_on, r_off, c_on, c_off = _on_off(ix, sp, prm)
    _same(r_on, r_off)
    assert c_on.postings == c_off.postings
    assert c_off.dense_postings == 0 and c_off.dense_reads == 0
    assert 0 < c_on.dense_postings < c_on.postings        # min_shared 4: up to two map probes per item
    assert c_on.dense_reads > 0
    oh, ost, og = db.search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
    assert r_on.hits["id"].tobytes() == oh["id"].tobytes()
    assert np.array_equal(r_on.stats["n_scored"], ost["n_scored"])
    assert np.array_equal(r_on.hist, og)
    assert c_on.postings == int(ost["pairs_total"].sum())


@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_dense_budget_of_one_count(open_db, schedule):
    """min_shared 3 leaves a budget of one count: an item reads at most one
    probe from a map and streams any other, and the filter's threshold drops
    to 2.  Results must equal the postings-only search and the oracle."""
    w, prot, sp, db = open_db
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(w.mods), w.max_mods, merge_tol=1).upload()
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, 3,
                               max_charge=3, schedule=schedule)
    _say(f"dense: min_shared 3, schedule {schedule}")
    r_on, r_off, c_on, c_off = _on_off(ix, sp, prm)
    _same(r_on, r_off)
    assert c_on.postings == c_off.postings and 0 < c_on.dense_postings < c_on.postings
    oh, ost, og = db.search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, 3)
    assert r_on.hits["id"].tobytes() == oh["id"].tobytes()
    assert np.array_equal(r_on.stats["n_scored"], ost["n_scored"])
    assert np.array_equal(r_on.hist, og)


@pytest.mark.parametrize("tile,threads,tpi", [(4096, 256, 1), (8192, 512, 3), (32768, 512, 2), (16384, 256, 5)])
def test_dense_with_schedules_and_item_edges(open_db, tile, threads, tpi):
    """Work items that start and end inside tiles, several candidate buffers
    per tile: every admitted id reads its own map bits."""
    w, prot, sp, db = open_db
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(w.mods), w.max_mods, merge_tol=1).upload()
    ix.set_schedule(tile=tile, group_threads=threads, tiles_per_item=tpi)
    _say(f"dense schedules: tile {tile}, threads {threads}, tiles per item {tpi}")
    for schedule in (capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT):
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k,
                                   w.min_shared, max_charge=3, schedule=schedule)
        r_on, r_off, _, _ = _on_off(ix, sp, prm)
        _same(r_on, r_off)


def test_dense_closed_search_parity():
    """Closed windows (10 ppm) cover a few ids inside one tile."""
    w = synth.workload("tiny")
    prot = w.proteome()
    sp = w.spectra(prot, n=400, seed=3)
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, [], 0).upload()
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, [], 0)
    assert ix.dense()[0].size >= 2
    for schedule in (capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT):
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                                   max_charge=2, schedule=schedule)
        _say(f"dense closed search: schedule {schedule}")
        r_on, r_off, c_on, _ = _on_off(ix, sp, prm)
        _same(r_on, r_off)
        assert c_on.dense_postings > 0
        oh, ost, og = db.search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
        assert r_on.hits["id"].tobytes() == oh["id"].tobytes()
        assert np.array_equal(r_on.hist, og)


def test_dense_wide_counters_and_many_dense_probes(open_db):
    """A spectrum with hundreds of peaks on a y1 bin and min_shared 7: more
    map probes fit the threshold than an item keeps (the rest are streamed),
    and counts past the narrow counter's fields (64-bit counters)."""
    w, prot, sp, db = open_db
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(w.mods), w.max_mods).upload()
    pid = 777
    b, y = oracle.ions(db.residue_masses(pid))
    y1_r = 175.11895                                   # R + H2O + H+: a dense list
    peaks = [(y1_r, 10.0)] * 230 + [(float(m) * 1e-6, 3.0) for m in np.concatenate([b, y])][:26]
    prec = (db.get(pid)[0] * 1e-6 + 2 * 1.007276) / 2
    sp1 = _mk([peaks, peaks[:30], peaks[200:]], [prec, prec, prec], [2, 3, 2])
    prm = engine.search_params(False, 500_000_000, 1, 256, 5, 7, max_charge=3)
    _say("dense: wide counters, many dense probes")
    r_on, r_off, c_on, _ = _on_off(ix, sp1, prm)
    _same(r_on, r_off)
    assert c_on.wide_spectra >= 1 and c_on.dense_postings > 0
    oh, ost, og = db.search(sp1, False, 500_000_000, 1, 256, 5, 7)
    assert r_on.hits["id"].tobytes() == oh["id"].tobytes()
    assert c_on.dense_reads > 0
    for f in ("n_b", "n_y", "sum_q"):
        assert np.array_equal(r_on.hits[f], oh[f]), f
    assert np.array_equal(r_on.hist, og)


def _mk(peak_lists, prec, charge):
    off = np.zeros(len(peak_lists) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in peak_lists])
    mz = np.array([m for p in peak_lists for m, _ in p], np.float32)
    it = np.array([i for p in peak_lists for _, i in p], np.float32)
    return synth.Spectra(off, mz, it, np.asarray(prec, np.float64), np.asarray(charge, np.int8))


def test_dense_maps_cover_lists_longer_than_one_grid():
    """A y1 list of the large open-search index (about 41 million peptides,
    merged lists) holds more postings than one capped launch grid has threads:
    the map must hold all of them.  Every scored candidate of the heaviest
    spectra, whose windows reach the last ids, must match the postings-only
    search."""
    w = synth.workload("large")
    prot = w.proteome()
    ix = engine.HostIndex.build_on_device(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                                          engine.mods_from_synth(w.mods), w.max_mods, merge_tol=w.frag_tol_bins)
    n_pep = len(ix)
    off = np.zeros(ix.shape()[2] + 1, np.uint64)        # bin offsets only (no postings to the host)
    capi.check(capi.ps_index_host_arrays(ix.handle, engine.ptr(off), None))
    bins, _ = ix.dense()
    longest = int(max(off[b + 1] - off[b] for b in bins.tolist()))
    _say(f"dense: large index, {n_pep} peptides, longest dense list {longest} postings")
    assert longest > 65536 * 256
    sp = w.spectra(prot, n=3000, seed=11)
    mass = (sp.precursor_mz - 1.007276) * sp.charge
    pick = np.argsort(-mass, kind="stable")[:4]
    sub = sp.subset(pick.tolist())
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=int(sub.charge.max()))
    dumps = {}
    for dense in (False, True):
        ix.set_dense(dense)
        try:
            dumps[dense] = engine.search_dump(ix, sub, prm)
        finally:
            ix.set_dense(True)
    ids = dumps[True][1]
    _say(f"dense: {ids.size} scored candidates, highest id {int(ids.max()) if ids.size else -1}")
    assert ids.size and int(ids.max()) > n_pep * 0.9
    for a, b in zip(dumps[True], dumps[False]):
        assert np.array_equal(a, b)
    r_on, r_off, c_on, _ = _on_off(ix, sub, prm)
    _same(r_on, r_off)
    assert c_on.dense_reads > 0

"""Parity of the HIP search path with the CPU oracle (needs an MI355X).

Integer outputs (window sizes, scored counts, top-k ids, n_b/n_y/S, histograms,
the full scored set) must be bit-exact.  Hyperscores come from the same fp64
table values on both sides, so they agree to the last bit; expect values go
through GPU log10/pow and a differently ordered sum, so they are held to 1e-5
relative.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2102_02286_amd import capi, engine, synth

pytestmark = pytest.mark.gpu

EV_RTOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def assert_parity(res, oh, ost, og, check_hist=True):
    assert res.hits.shape == oh.shape
    bad = np.nonzero(np.any(res.hits["id"] != oh["id"], axis=1))[0]
    assert bad.size == 0, f"top-k ids differ for spectra {bad[:10]}"
    for f in ("n_b", "n_y", "sum_q"):
        assert np.array_equal(res.hits[f], oh[f]), f
    h1, h2 = res.hits["hyperscore"], oh["hyperscore"]
    assert np.array_equal(np.isinf(h1), np.isinf(h2))
    fin = np.isfinite(h2)
    assert np.array_equal(h1[fin], h2[fin])
    for f in ("n_window", "n_scored", "status"):
        assert np.array_equal(res.stats[f].astype(np.int64), ost[f].astype(np.int64)), f
    ok = ost["status"] == 0
    assert np.all(np.isnan(res.stats["evalue"][~ok]))
    np.testing.assert_allclose(res.stats["evalue"][ok], ost["evalue"][ok], rtol=EV_RTOL)
    if check_hist:
        assert np.array_equal(res.hist, og)


# ---------------------------------------------------------------------------
# tiny closed search: the whole 1000-spectrum batch
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def tiny():
    w = synth.workload("tiny")
    prot = w.proteome()
    sp = w.spectra(prot)
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, [], 0).upload()
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, [], 0)
    return w, prot, sp, ix, db


@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_tiny_full_batch_parity(tiny, schedule):
    w, prot, sp, ix, db = tiny
    _say(f"tiny: {sp.n} spectra, schedule {schedule}")
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=2, schedule=schedule)
    res = engine.search(ix, sp, prm)
    oh, ost, og = db.search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
    assert_parity(res, oh, ost, og)
    assert res.postings == int(ost["pairs_total"].sum())


class _OneCallIndex:
    """An index from ps_build_index and the device block it lives in."""

    def __init__(self, handle, arena):
        self.handle, self.arena = handle, arena

    def __del__(self):
        if self.handle is not None and self.handle.value:
            capi.ps_index_free(self.handle)
            self.handle = None


def test_one_call_build_equals_create_and_upload(tiny):
    """ps_build_index (the index created and uploaded in one call) searches
    exactly as ps_index_create + ps_index_upload, and as the oracle; a block
    one byte too small is refused and leaves no index."""
    import torch
    w, prot, sp, ix, db = tiny
    p, keep = engine._db_params(w.missed, w.min_len, w.max_len, [], 0)
    res = np.ascontiguousarray(prot.residues, dtype=np.uint8)
    off = np.ascontiguousarray(prot.offsets, dtype=np.uint64)
    need = C.c_uint64()
    capi.check(capi.ps_index_device_bytes(ix.handle, C.byref(need)))
    arena = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    small = capi.ps_device(arena.data_ptr(), need.value - 1, st)
    h = C.c_void_p()
    _say("one-call build: a block one byte short")
    assert capi.ps_build_index(C.byref(small), C.byref(p), capi.ptr(res), capi.ptr(off), off.shape[0] - 1,
                               C.byref(h)) == capi.PS_ENOMEM
    assert not h.value
    dev = capi.ps_device(arena.data_ptr(), arena.numel(), st)
    _say("one-call build")
    capi.check(capi.ps_build_index(C.byref(dev), C.byref(p), capi.ptr(res), capi.ptr(off), off.shape[0] - 1,
                                   C.byref(h)), "ps_build_index")
    one = _OneCallIndex(h, arena)
    assert engine.HostIndex.shape(one) == ix.shape()
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=2)
    r1, r0 = engine.search(one, sp, prm), engine.search(ix, sp, prm)
    assert r1.hits.tobytes() == r0.hits.tobytes() and r1.hist.tobytes() == r0.hist.tobytes()
    oh, ost, og = db.search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
    assert_parity(r1, oh, ost, og)


def test_tiny_scored_set_dump(tiny):
    w, prot, sp, ix, db = tiny
    sub = sp.subset(np.arange(0, 200))
    _say("tiny: scored-set dump, 200 spectra")
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, 1, max_charge=2)
    gs, gi, gb, gy, gq = engine.search_dump(ix, sub, prm)
    want = []
    for s in range(sub.n):
        ids, nb, ny, sq = db.scored(sub, s, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, min_shared=1)
        want += [(s, int(a), int(b), int(c), int(d)) for a, b, c, d in zip(ids, nb, ny, sq)]
    got = list(zip(gs.tolist(), gi.tolist(), gb.tolist(), gy.tolist(), gq.tolist()))
    assert got == want


# ---------------------------------------------------------------------------
# open search on a small proteome: many tiles per window, ragged tails
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_open():
    w = synth.workload("medium")
    prot = synth.make_proteome(2000, seed=0)
    sp = w.spectra(prot, n=160, seed=5)
    mods = w.mods
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(mods), w.max_mods).upload()
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                         oracle.mods_from_synth(mods), w.max_mods)
    oh, ost, og = db.search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
    return w, prot, sp, ix, db, (oh, ost, og)


def test_small_open_search_parity(small_open):
    w, prot, sp, ix, db, (oh, ost, og) = small_open
    _say(f"small open: {len(db)} peptides, {sp.n} spectra")
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3)
    res = engine.search(ix, sp, prm)
    assert (ost["n_window"] > 4 * 8192).sum() > 50          # windows span several LDS tiles
    assert_parity(res, oh, ost, og)
    assert res.postings == int(ost["pairs_total"].sum())


def test_small_open_scored_set_dump(small_open):
    w, prot, sp, ix, db, _ = small_open
    sub = sp.subset(np.arange(0, 12))
    _say("small open: scored-set dump, 12 spectra")
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3)
    gs, gi, gb, gy, gq = engine.search_dump(ix, sub, prm)
    want = []
    for s in range(sub.n):
        ids, nb, ny, sq = db.scored(sub, s, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks,
                                    min_shared=w.min_shared)
        want += [(s, int(a), int(b), int(c), int(d)) for a, b, c, d in zip(ids, nb, ny, sq)]
    got = list(zip(gs.tolist(), gi.tolist(), gb.tolist(), gy.tolist(), gq.tolist()))
    assert got == want


def test_small_open_permutation_and_split_invariance(small_open):
    w, prot, sp, ix, db, _ = small_open
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3)
    _say("small open: permutation / split invariance")
    r0 = engine.search(ix, sp, prm)
    perm = np.random.default_rng(7).permutation(sp.n)
    r1 = engine.search(ix, sp.subset(perm), prm)
    assert r1.hits.tobytes() == r0.hits[perm].tobytes()
    assert r1.stats.tobytes() == r0.stats[perm].tobytes()
    ra = engine.search(ix, sp.subset(np.arange(0, 70)), prm)
    rb = engine.search(ix, sp.subset(np.arange(70, sp.n)), prm)
    assert np.concatenate([ra.hits, rb.hits]).tobytes() == r0.hits.tobytes()
    assert np.concatenate([ra.stats, rb.stats]).tobytes() == r0.stats.tobytes()
    # the same batch twice: bit-identical
    r2 = engine.search(ix, sp, prm)
    assert r2.hits.tobytes() == r0.hits.tobytes() and r2.hist.tobytes() == r0.hist.tobytes()


def _protein_order(prot, perm):
    seqs = [prot.residues[int(prot.offsets[i]):int(prot.offsets[i + 1])] for i in range(len(prot.offsets) - 1)]
    off = np.zeros(len(perm) + 1, np.uint64)
    off[1:] = np.cumsum([len(seqs[i]) for i in perm])
    return np.concatenate([seqs[i] for i in perm]).astype(np.uint8), off


def _entry_keys(ents, residues, offsets):
    a = offsets[ents["prot"].astype(np.int64)].astype(np.int64) + ents["start"].astype(np.int64)
    return [(bytes(residues[x:x + int(n)]), int(st) == 0, int(m))
            for x, n, st, m in zip(a, ents["len"], ents["start"], ents["mask"])]


def test_small_open_protein_order_invariance(small_open):
    """Reordering the proteins renumbers the peptides but changes no spectrum's
    scored set (as peptides with their counts), statistics or histogram."""
    from collections import Counter
    w, prot, sp, ix, db, _ = small_open
    res2, off2 = _protein_order(prot, np.random.default_rng(11).permutation(len(prot.offsets) - 1))
    ix2 = engine.HostIndex(res2, off2, w.missed, w.min_len, w.max_len, engine.mods_from_synth(w.mods),
                           w.max_mods).upload()
    assert len(ix2) == len(ix)
    _say("small open: protein-order invariance")
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3)
    r1, r2 = engine.search(ix, sp, prm), engine.search(ix2, sp, prm)
    assert r1.stats.tobytes() == r2.stats.tobytes()
    assert r1.hist.tobytes() == r2.hist.tobytes()
    assert r1.hits["hyperscore"].tobytes() == r2.hits["hyperscore"].tobytes()
    k1 = _entry_keys(ix.entries(), prot.residues, prot.offsets)
    k2 = _entry_keys(ix2.entries(), res2, off2)
    sets = []
    for index, keys in ((ix, k1), (ix2, k2)):
        gs, gi, gb, gy, gq = engine.search_dump(index, sp, prm)
        sets.append(Counter((int(s), keys[int(i)], int(b), int(y), int(q)) for s, i, b, y, q in zip(gs, gi, gb, gy, gq)))
    assert sets[0] == sets[1] and len(sets[0]) > 0


@pytest.mark.parametrize("sched", [dict(tile=4096), dict(tile=8192), dict(tile=16384), dict(tile=32768),
                                   dict(tile=8192, group_threads=512), dict(tile=32768, group_threads=512)])
def test_schedules_give_identical_results(small_open, sched):
    """The tile size and the workgroup size change only speed."""
    w, prot, sp, ix, db, (oh, ost, og) = small_open
    assert ix.directory()[0] == 12
    old = ix.schedule()
    try:
        ix.set_schedule(**sched)
        _say(f"schedule {sched}")
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                                   max_charge=3)
        res = engine.search(ix, sp, prm)
        assert_parity(res, oh, ost, og)
        assert res.postings == int(ost["pairs_total"].sum())
    finally:
        capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(old)))


@pytest.mark.parametrize("sched", [dict(tiles_per_item=1), dict(tiles_per_item=3, tile=8192),
                                   dict(tiles_per_item=64, groups_per_cu=1), dict(tiles_per_item=5, groups_per_cu=8),
                                   dict(tiles_per_item=2, tile=8192, group_threads=512),
                                   dict(tiles_per_item=9, tile=16384, group_threads=512, groups_per_cu=3)])
def test_persistent_schedule_parity(small_open, sched):
    """The work-queue scan splits windows into (spectrum, tile range) items;
    merged results equal the oracle for any item size."""
    w, prot, sp, ix, db, (oh, ost, og) = small_open
    old = ix.schedule()
    try:
        ix.set_schedule(**sched)
        _say(f"persistent {sched}")
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                                   max_charge=3, schedule=capi.PS_SCHED_PERSISTENT)
        res = engine.search(ix, sp, prm)
        assert_parity(res, oh, ost, og)
        assert res.postings == int(ost["pairs_total"].sum())
    finally:
        capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(old)))


def test_plan_graph_replays_match_eager_and_oracle(small_open):
    """One captured graph, replayed for batches of different sizes with eager
    searches and synchronisations in between; every replay equals the eager
    result and the oracle."""
    import torch
    w, prot, sp, ix, db, (oh, ost, og) = small_open
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=capi.PS_SCHED_PERSISTENT)
    plan = engine.Plan(ix, prm, n_cap=sp.n, nnz_cap=int(sp.peak_off[-1]))
    own = C.c_void_p()
    capi.check(capi.ps_plan_stream(plan.handle, C.byref(own)))
    assert own.value                                   # no stream given: the plan made its own
    given = torch.cuda.Stream()                        # default priority
    plan_on = engine.Plan(ix, prm, n_cap=4, nnz_cap=int(sp.peak_off[4]), stream=given)
    got_on = C.c_void_p()
    capi.check(capi.ps_plan_stream(plan_on.handle, C.byref(got_on)))
    assert got_on.value == given.cuda_stream
    del plan_on
    ranges = [(0, sp.n), (10, 50), (0, 1), (100, sp.n), (0, sp.n), (33, 34)]
    for k, (a, b) in enumerate(ranges):
        sub = sp.subset(np.arange(a, b))
        _say(f"plan replay {k}: spectra [{a}, {b})")
        got = plan.search(sub)
        eager = engine.search(ix, sub, prm)
        torch.cuda.synchronize()
        assert got.hits.tobytes() == eager.hits.tobytes()
        assert got.stats.tobytes() == eager.stats.tobytes()
        assert got.hist.tobytes() == eager.hist.tobytes()
        from types import SimpleNamespace
        assert_parity(SimpleNamespace(hits=got.hits, stats=got.stats, hist=got.hist), oh[a:b], ost[a:b], og[a:b])


class _DevArray:
    """A raw device buffer seen by torch (no copy)."""

    def __init__(self, p, n, typestr):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (p, False), "version": 2}


def test_plan_device_inputs(small_open):
    import torch
    w, prot, sp, ix, db, (oh, ost, og) = small_open
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=capi.PS_SCHED_PERSISTENT)
    nnz = int(sp.peak_off[-1])
    plan = engine.Plan(ix, prm, n_cap=sp.n, nnz_cap=nnz)
    d = plan.inputs()
    pairs = [(d.peak_off, sp.peak_off.astype(np.uint64).view(np.int64), "<i8"), (d.mz, sp.mz, "<f4"),
             (d.intensity, sp.intensity, "<f4"), (d.precursor_mz, sp.precursor_mz, "<f8"), (d.charge, sp.charge, "|i1")]
    for p, host, ts in pairs:
        dst = torch.as_tensor(_DevArray(p, host.shape[0], ts), device="cuda")
        dst.copy_(torch.from_numpy(np.ascontiguousarray(host)).to("cuda"))
    torch.cuda.synchronize()
    _say("plan with device inputs")
    plan.run_device(sp.n, nnz)
    got = plan.results()
    from types import SimpleNamespace
    assert_parity(SimpleNamespace(hits=got.hits, stats=got.stats, hist=got.hist), oh, ost, og)


def test_autotune_keeps_results_and_caches(small_open, tmp_path):
    w, prot, sp, ix, db, (oh, ost, og) = small_open
    old = ix.schedule()
    try:
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                                   max_charge=3, schedule=capi.PS_SCHED_PERSISTENT)
        cache = str(tmp_path / "tune.txt")
        _say("autotune")
        best, trials = engine.autotune(ix, sp.subset(np.arange(0, 60)), prm, cache_path=cache)
        assert len(trials) >= 5
        res = engine.search(ix, sp, prm)
        assert_parity(res, oh, ost, og)
        # a second call finds the cached schedule and measures nothing
        capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(old)))
        best2, trials2 = engine.autotune(ix, sp.subset(np.arange(0, 60)), prm, cache_path=cache)
        assert trials2 == [] and bytes(best2) == bytes(best)
        assert bytes(ix.schedule()) == bytes(best)
    finally:
        capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(old)))


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def _mk(peak_lists, prec, charges):
    off = np.zeros(len(peak_lists) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in peak_lists])
    mz = np.array([m for pl in peak_lists for (m, _) in pl], np.float32)
    it = np.array([i for pl in peak_lists for (_, i) in pl], np.float32)
    return synth.Spectra(off, mz, it, np.asarray(prec, np.float64), np.asarray(charges, np.int8))


def test_edge_cases_parity(small_open):
    w, prot, sp, ix, db, _ = small_open
    rng = np.random.default_rng(11)
    tab_mass = [db.get(int(i))[0] for i in rng.integers(0, len(db), 8)]
    b, y = oracle.ions(db.residue_masses(int(rng.integers(0, len(db)))))
    one_ion = float(b[2]) * 1e-6
    cases = [
        ([], 800.0, 2),                                                       # no peaks
        ([(500.0, 0.0), (600.0, 0.0)], 700.0, 2),                             # zero intensities
        ([(one_ion, 5.0)] * 120, (tab_mass[0] * 1e-6 + 2 * 1.007276) / 2, 2),  # duplicates: wide counters
        ([(one_ion + 0.001 * k, 1.0 + k % 3) for k in range(100)], 900.0, 3),  # crowded bins, intensity ties
        ([(float(m) * 1e-6, 1.0) for m in np.concatenate([b, y])], 650.5, 1),  # charge 1
        ([(float(m) * 1e-6, 2.0) for m in b], 410.25, 8),                     # charge 8 (7 fragment charges)
        ([(300.0, 1.0)], 20000.0, 2),                                         # window beyond every peptide
        ([(300.0 + k, 1.0) for k in range(300)], 1200.0, 3),                  # more peaks than top_peaks
    ]
    sp_e = _mk([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases])
    for top_k, kmin, T, top_b, window, ppm in [(1, 1, 1, 90, 500_000_000, False), (16, 2, 0, 90, 100_000_000, False),
                                               (5, 4, 4, 20, 500_000_000, False), (3, 1, 2, 50, 30, True),
                                               (5, 1, 1, 90, 10**15, False)]:
        for fit in (capi.PS_FIT_TAIL, capi.PS_FIT_GUMBEL):
            _say(f"edge: top_k={top_k} kmin={kmin} T={T} B={top_b} window={window} ppm={ppm} fit={fit}")
            prm = engine.search_params(ppm, window, T, top_b, top_k, kmin,
                                       max_charge=8 if (2 * T + 1) * 7 * top_b <= 2048 else 3, fit=fit)
            sub = sp_e if prm.max_charge == 8 else sp_e.subset([i for i in range(sp_e.n) if sp_e.charge[i] <= 3])
            res = engine.search(ix, sub, prm)
            oh, ost, og = db.search(sub, ppm, window, T, top_b, top_k, kmin, fit=fit)
            assert_parity(res, oh, ost, og)


@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_spectra_with_many_peaks_parity(small_open, schedule):
    """Spectra with more peaks than the prep stages in LDS (up to the 4096
    allowed), with intensity ties broken by m/z and by input order, next to
    small ones: top-B selection and everything after it against the oracle."""
    w, prot, sp, ix, db, _ = small_open
    rng = np.random.default_rng(21)
    lists, prec, ch = [], [], []
    for n_peaks in (1023, 1024, 1025, 2000, 4096, 60):
        pid = int(rng.integers(0, len(db)))
        b, y = oracle.ions(db.residue_masses(pid))
        ions = [float(m) * 1e-6 for m in np.concatenate([b, y])]
        mz = np.concatenate([ions, rng.uniform(150.0, 2000.0, max(0, n_peaks - len(ions)))])[:n_peaks]
        inten = rng.integers(1, 40, n_peaks).astype(np.float64)      # many equal intensities
        inten[:min(len(ions), n_peaks)] += 20.0                       # the true ions among the strongest
        mz[5::97] = mz[4::97][:len(mz[5::97])]                        # equal m/z and intensity: input order decides
        inten[5::97] = inten[4::97][:len(inten[5::97])]
        lists.append(list(zip(mz.tolist(), inten.tolist())))
        prec.append((db.get(pid)[0] * 1e-6 + 2 * 1.007276) / 2)
        ch.append(2 + (n_peaks % 2))
    sp_m = _mk(lists, prec, ch)
    for top_b, noise, inten_mode in ((100, 0, capi.PS_INTENSITY_LINEAR), (256, 50, capi.PS_INTENSITY_SQRT)):
        _say(f"many peaks: schedule {schedule}, B={top_b}, noise {noise}, intensity {inten_mode}")
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, top_b, w.top_k, w.min_shared,
                                   max_charge=3, schedule=schedule, noise_permille=noise, intensity=inten_mode)
        res = engine.search(ix, sp_m, prm)
        oh, ost, og = db.search(sp_m, w.window_is_ppm, w.window, w.frag_tol_bins, top_b, w.top_k, w.min_shared,
                                noise_permille=noise, intensity=oracle.INTENSITY_SQRT if inten_mode else
                                oracle.INTENSITY_LINEAR)
        assert_parity(res, oh, ost, og)
        assert (ost["status"] == 0).sum() >= 5


def test_wide_counters_are_used_and_exact(small_open):
    """A spectrum whose peaks pile into one bin needs 64-bit counters; the
    result must still equal the oracle's unbounded counts."""
    w, prot, sp, ix, db, _ = small_open
    pid = 1234
    b, y = oracle.ions(db.residue_masses(pid))
    ion = float(y[0]) * 1e-6
    peaks = [(ion, 10.0)] * 256                       # 256 shared y pairs: past an 8-bit field
    sp1 = _mk([peaks], [(db.get(pid)[0] * 1e-6 + 2 * 1.007276) / 2], [2])
    prm = engine.search_params(False, 500_000_000, 1, 256, 5, 1, max_charge=2)
    _say("wide counters")
    res = engine.search(ix, sp1, prm)
    oh, ost, og = db.search(sp1, False, 500_000_000, 1, 256, 5, 1)
    assert int(oh["n_y"][0, 0]) > 255
    assert_parity(res, oh, ost, og)


def test_device_resident_inputs_and_invalid_spectra(small_open):
    import torch
    w, prot, sp, ix, db, _ = small_open
    sub = sp.subset(np.arange(0, 40))
    charge = sub.charge.copy()
    charge[3] = 0                       # invalid charge
    prec = sub.precursor_mz.copy()
    prec[5] = np.nan                    # invalid precursor
    mz = sub.mz.copy()
    mz[int(sub.peak_off[7])] = -1.0     # invalid peak
    dev = "cuda:0"
    t = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in
         (sub.peak_off.astype(np.uint64).view(np.int64), mz, sub.intensity, prec, charge)]
    s = capi.ps_spectra(sub.n, *[x.data_ptr() for x in t])
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3)
    import ctypes as C
    need = C.c_uint64()
    capi.check(capi.ps_workspace_bytes(ix.handle, sub.n, int(sub.peak_off[-1]), C.byref(prm), C.byref(need)))
    ws = engine.Workspace()
    d = ws.get(need.value)
    bh = C.c_void_p()
    _say("device-resident inputs")
    capi.check(capi.ps_search_device(ix.handle, C.byref(d), C.byref(s), int(sub.peak_off[-1]), C.byref(prm),
                                     C.byref(bh)))
    res = engine.collect(bh, sub.n, prm)
    capi.ps_batch_free(bh)
    st = res.stats["status"]
    assert st[3] == capi.PS_STATUS_INVALID and st[5] == capi.PS_STATUS_INVALID and st[7] == capi.PS_STATUS_INVALID
    good = np.array([i for i in range(sub.n) if i not in (3, 5, 7)])
    ref = engine.search(ix, sub.subset(good), prm)
    assert res.hits[good].tobytes() == ref.hits.tobytes()
    assert res.stats[good].tobytes() == ref.stats.tobytes()
    # the host path rejects the same batch outright
    sp_bad = synth.Spectra(sub.peak_off, mz, sub.intensity, prec, charge)
    with pytest.raises(capi.PsError) as e:
        engine.search(ix, sp_bad, prm)
    assert e.value.code == capi.PS_EINVAL


# ---------------------------------------------------------------------------
# full-size medium workload: sampled outputs against the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_medium_full_size_sampled_parity(schedule):
    w = synth.workload("medium")
    prot = w.proteome()
    _say("medium: building index")
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(w.mods), w.max_mods).upload()
    sp = w.spectra(prot)
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=schedule)
    _say(f"medium: searching {sp.n} spectra, schedule {schedule}")
    res = engine.search(ix, sp, prm)
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                         oracle.mods_from_synth(w.mods), w.max_mods)
    idx = np.sort(np.random.default_rng(123).choice(sp.n, 24, replace=False))
    sub = sp.subset(idx)
    _say("medium: oracle on 24 sampled spectra")
    oh, ost, og = db.search(sub, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
    from types import SimpleNamespace
    part = SimpleNamespace(hits=res.hits[idx], stats=res.stats[idx], hist=res.hist[idx])
    assert_parity(part, oh, ost, og)


def test_dense_tiles_use_several_map_chunks(small_open):
    """Spectra whose peaks sit on the densest fragment bins (b1 and y1 of every
    residue): with 32768-candidate tiles a tile holds more than 8192 postings,
    so its postings are mapped to probes in several chunks."""
    from tests import bruteforce as bf
    w, prot, sp, ix, db, _ = small_open
    H, W = bf.PROTON_UDA, bf.WATER_UDA
    letters = "GASPVTCLINDQKEMHFRYW"
    peaks = [((bf.RES_UDA[c] + H) * 1e-6, 50.0 + i) for i, c in enumerate(letters)]
    peaks += [((bf.RES_UDA[c] + W + H) * 1e-6, 80.0 + i) for i, c in enumerate(letters)]
    lists = [peaks, peaks[::2], peaks[1::2] + peaks[:5]]
    prec = [(1400.0 + 1.007276 * 2) / 2, (1700.0 + 1.007276 * 2) / 2, (1100.0 + 1.007276 * 2) / 2]
    off = np.zeros(len(lists) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in lists])
    dense = synth.Spectra(off, np.array([m for p in lists for m, _ in p], np.float32),
                          np.array([v for p in lists for _, v in p], np.float32), np.array(prec, np.float64),
                          np.array([2, 2, 2], np.int8))
    tol = 2
    oh, ost, og = db.search(dense, w.window_is_ppm, w.window, tol, w.top_peaks, w.top_k, w.min_shared)
    # postings per 32768-candidate tile of the first spectrum, counted on the host
    boff, post = ix.host_arrays()
    ids = post >> 1
    lo, hi = int(ost["lo"][0]), int(ost["hi"][0])
    per_tile = np.zeros((hi >> 15) + 1, np.int64)
    for m, _ in peaks:
        b = int((int(round(float(np.float32(m)) * 1e6)) + 5000) // 10000)
        for d in range(-tol, tol + 1):
            r = ids[boff[b + d]:boff[b + d + 1]]
            r = r[(r >= lo) & (r < hi)]
            np.add.at(per_tile, r >> 15, 1)
    assert per_tile.max() > 8192, per_tile.max()
    old = ix.schedule()
    try:
        for sched in (dict(tile=32768), dict(tile=4096)):
            for schedule in (capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT):
                ix.set_schedule(**sched)
                _say(f"dense tiles {sched} schedule {schedule}")
                prm = engine.search_params(w.window_is_ppm, w.window, tol, w.top_peaks, w.top_k, w.min_shared,
                                           max_charge=3, schedule=schedule)
                res = engine.search(ix, dense, prm)
                assert_parity(res, oh, ost, og)
                assert res.postings == int(ost["pairs_total"].sum())
    finally:
        capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(old)))


# ---------------------------------------------------------------------------
# indexes whose lists merge the 2T+1 neighbouring bins: one probe per peak
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_tiny_merged_lists_parity(tiny, schedule):
    w, prot, sp, _, db = tiny
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, [], 0,
                          merge_tol=w.frag_tol_bins).upload()
    _say(f"tiny merged T={w.frag_tol_bins}: {sp.n} spectra, schedule {schedule}")
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=2, schedule=schedule)
    res = engine.search(ix, sp, prm)
    oh, ost, og = db.search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
    assert_parity(res, oh, ost, og)
    assert res.postings == int(ost["pairs_total"].sum())
    sub = sp.subset(np.arange(0, 100))
    prm1 = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, 1, max_charge=2)
    gs, gi, gb, gy, gq = engine.search_dump(ix, sub, prm1)
    want = []
    for s in range(sub.n):
        ids, nb, ny, sq = db.scored(sub, s, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, min_shared=1)
        want += [(s, int(a), int(b), int(c), int(d)) for a, b, c, d in zip(ids, nb, ny, sq)]
    assert list(zip(gs.tolist(), gi.tolist(), gb.tolist(), gy.tolist(), gq.tolist())) == want


@pytest.fixture(scope="module")
def small_open_merged(small_open):
    w, prot, sp, _, db, expect = small_open
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(w.mods), w.max_mods, merge_tol=w.frag_tol_bins).upload()
    return w, prot, sp, ix, db, expect


@pytest.mark.parametrize("sched", [dict(tile=4096, tiles_per_item=64), dict(tile=8192, tiles_per_item=3),
                                   dict(tile=4096, tiles_per_item=1, groups_per_cu=8),
                                   dict(tile=8192, tiles_per_item=2, group_threads=512)])
@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_small_open_merged_lists_parity(small_open_merged, sched, schedule):
    w, prot, sp, ix, db, (oh, ost, og) = small_open_merged
    ix.set_schedule(**{"group_threads": 0, **sched})
    _say(f"small open merged: {sched} schedule {schedule}")
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=schedule)
    res = engine.search(ix, sp, prm)
    assert_parity(res, oh, ost, og)
    assert res.postings == int(ost["pairs_total"].sum())


@pytest.mark.parametrize("noise,inten", [(150, capi.PS_INTENSITY_LINEAR), (0, capi.PS_INTENSITY_SQRT),
                                         (400, capi.PS_INTENSITY_SQRT), (1000, capi.PS_INTENSITY_LINEAR)])
def test_preprocessing_variants_parity(small_open, noise, inten):
    """Noise clearing before the top-B selection and square-root intensities,
    against the oracle with the same options (both schedules)."""
    w, prot, sp, ix, db, _ = small_open
    sub = sp.subset(np.arange(0, 64))
    oh, ost, og = db.search(sub, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                            noise_permille=noise, intensity=inten)
    for schedule in (capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT):
        _say(f"pre-processing: noise {noise} intensity {inten} schedule {schedule}")
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                                   max_charge=3, schedule=schedule, noise_permille=noise, intensity=inten)
        res = engine.search(ix, sub, prm)
        assert_parity(res, oh, ost, og)
        assert res.postings == int(ost["pairs_total"].sum())


@pytest.mark.parametrize("types,T", [(63, 1), (4 | 32, 2)])
def test_other_ion_series_parity(types, T):
    """Indexes of the a, c, x and z series (N-terminal matches in n_b,
    C-terminal in n_y) against the oracle with the same series, both schedules."""
    w = synth.workload("medium")
    prot = synth.make_proteome(600, seed=2)
    sp = w.spectra(prot, n=48, seed=8)
    mods = [synth.OXIDATION, synth.ACETYL_NTERM]
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, engine.mods_from_synth(mods),
                          2, merge_tol=T, ion_types=types).upload()
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, oracle.mods_from_synth(mods), 2)
    oh, ost, og = db.search(sp, False, 300_000_000, T, w.top_peaks, w.top_k, 3, ion_types=types)
    assert (ost["status"] == 0).sum() > 20
    for schedule in (capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT):
        _say(f"ion series {types}, merge {T}, schedule {schedule}")
        prm = engine.search_params(False, 300_000_000, T, w.top_peaks, w.top_k, 3, max_charge=3, schedule=schedule)
        res = engine.search(ix, sp, prm)
        assert_parity(res, oh, ost, og)
        assert res.postings == int(ost["pairs_total"].sum())


def test_negative_zero_intensities_parity(small_open):
    """-0.0 is a valid intensity equal to 0: it must neither become the most
    intense peak nor change q, the noise cut or the top-B order."""
    w, prot, sp, ix, db, _ = small_open
    base = sp.subset(np.arange(0, 24))
    inten = base.intensity.copy()
    inten[::3] = -0.0
    inten[1::7] = 0.0
    sp0 = synth.Spectra(base.peak_off, base.mz, inten, base.precursor_mz, base.charge)
    assert np.signbit(sp0.intensity).sum() > 0
    for noise in (0, 200):
        _say(f"-0.0 intensities, noise {noise}")
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                                   max_charge=3, noise_permille=noise)
        res = engine.search(ix, sp0, prm)
        oh, ost, og = db.search(sp0, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                                noise_permille=noise)
        assert_parity(res, oh, ost, og)
        # and the same as writing +0.0
        pos = synth.Spectra(base.peak_off, base.mz, np.abs(inten), base.precursor_mz, base.charge)
        rp = engine.search(ix, pos, prm)
        assert rp.hits.tobytes() == res.hits.tobytes() and rp.stats.tobytes() == res.stats.tobytes()


def test_top_hit_in_the_open_histogram_bin_parity():
    """A 40-residue peptide matched on every b and y ion scores past 51.1: the
    hit lands in the open bin 511 and the tail fit stops at bin 510, on the GPU
    as in the oracle."""
    from tests import bruteforce as bf
    pep = "GASPVTCLINDQEMHFYWGASPVTCLINDQEMHFYWGAGK"
    rng = np.random.default_rng(51)
    filler = "".join(rng.choice(list("GASPVTLINDQEMHFYWKR"), 3000))
    proteins = [pep + "R" + filler[:1500], filler[1500:]]
    res_arr = np.frombuffer("".join(proteins).encode(), dtype=np.uint8)
    off = np.zeros(len(proteins) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in proteins])
    db = oracle.Database(res_arr, off, 1, 4, 45, [], 0)
    pid = [i for i in range(len(db)) if db.get(i)[1:4] == (0, 0, 40)][0]
    b, y = oracle.ions(db.residue_masses(pid))
    peaks = [(float(m) * 1e-6, 10.0) for m in np.concatenate([b, y])]
    peaks += [(float(rng.uniform(100, 2000)), float(rng.lognormal())) for _ in range(40)]
    sp1 = _mk([peaks, peaks[::2]], [(db.get(pid)[0] * 1e-6 + 2 * bf.PROTON_UDA * 1e-6) / 2] * 2, [2, 2])
    for T in (0, 1):
        ix = engine.HostIndex(res_arr, off, 1, 4, 45, [], 0, merge_tol=T).upload()
        for schedule in (capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT):
            for fit in (capi.PS_FIT_TAIL, capi.PS_FIT_GUMBEL):
                _say(f"open bin: merge {T} schedule {schedule} fit {fit}")
                prm = engine.search_params(False, 10**12, T, 200, 5, 1, max_charge=2, schedule=schedule, fit=fit)
                res = engine.search(ix, sp1, prm)
                oh, ost, og = db.search(sp1, False, 10**12, T, 200, 5, 1, fit=fit)
                assert oh["hyperscore"][0, 0] > 51.1 and og[0, 511] >= 1
                assert_parity(res, oh, ost, og)


def test_counter_bound_overflow_is_reported():
    """256 copies of one peak at precursor charge 8 (seven fragment charges,
    so every charge's 256 entries share a bin) on an index of all six ion
    series: the worst-case shared pairs (1792 entries x 3 series per terminus)
    times 200 pass the 2^20 entries of the log10 S table, so the spectrum is
    reported as PS_STATUS_OVERFLOW with no hits (never a saturated count) and
    ps_results returns PS_EOVERFLOW.  The other spectra of the batch are
    unaffected."""
    w = synth.workload("medium")
    prot = synth.make_proteome(300, seed=4)
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, [], 0, ion_types=63).upload()
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, [], 0)
    normal = w.spectra(prot, n=6, seed=12)
    crafted = [[(500.0, 7.0)] * 256]
    lists = [list(zip(normal.mz[int(normal.peak_off[i]):int(normal.peak_off[i + 1])].tolist(),
                      normal.intensity[int(normal.peak_off[i]):int(normal.peak_off[i + 1])].tolist()))
             for i in range(normal.n)]
    sp_o = _mk(lists[:3] + crafted + lists[3:], list(normal.precursor_mz[:3]) + [400.0] +
               list(normal.precursor_mz[3:]), list(normal.charge[:3]) + [8] + list(normal.charge[3:]))
    prm = engine.search_params(False, 500_000_000, 0, 256, 5, 4, max_charge=8)
    import ctypes as C
    s, keep = engine._spectra_struct(sp_o)
    need = C.c_uint64()
    capi.check(capi.ps_workspace_bytes(ix.handle, sp_o.n, int(sp_o.peak_off[-1]), C.byref(prm), C.byref(need)))
    ws = engine.Workspace()
    d = ws.get(need.value)
    bh = C.c_void_p()
    _say("counter-bound overflow")
    capi.check(capi.ps_search_batch(ix.handle, C.byref(d), C.byref(s), C.byref(prm), C.byref(bh)))
    hits = np.zeros(sp_o.n * 5, capi.HIT_DTYPE)
    stats = np.zeros(sp_o.n, capi.STAT_DTYPE)
    hist = np.zeros(sp_o.n * 512, np.int32)
    rc = capi.ps_results(bh, engine.ptr(hits), engine.ptr(stats), engine.ptr(hist))
    capi.ps_batch_free(bh)
    assert rc == capi.PS_EOVERFLOW and "counter" in capi.last_error()
    assert stats["status"][3] == capi.PS_STATUS_OVERFLOW
    assert stats["n_scored"][3] == 0 and np.all(hits.reshape(-1, 5)[3]["id"] == 0xFFFFFFFF)
    assert np.isnan(stats["evalue"][3])
    # the rest equals the oracle on the same index series
    keep_idx = [0, 1, 2, 4, 5, 6]
    oh, ost, og = db.search(sp_o.subset(keep_idx), False, 500_000_000, 0, 256, 5, 4, ion_types=63)
    from types import SimpleNamespace
    part = SimpleNamespace(hits=hits.reshape(-1, 5)[keep_idx], stats=stats[keep_idx],
                           hist=hist.reshape(-1, 512)[keep_idx])
    assert_parity(part, oh, ost, og)

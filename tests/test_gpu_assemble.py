"""Result assembly over database partitions on the GPU (Superstep 4; needs an MI355X).

Every partition of a round-robin partitioned database (ps_db_params.n_shards,
.shard) is searched by the HIP path, and ps_assemble merges the partition
results on the device.  The assembled results must equal the whole-database
GPU search bit for bit, and the oracle's whole-database search to the parity
bar of the search itself (integers exact, expect values 1e-5 relative).
"""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2102_02286_amd import capi, engine, synth
from tests.test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _same(a, b):
    return a.tobytes() == b.tobytes()


def _assert_identical(r, ref):
    assert _same(r.hits, ref.hits), "hits differ"
    assert _same(r.stats, ref.stats), "stats differ"
    assert _same(r.hist, ref.hist), "histograms differ"


def _index(prot, w, merge_tol, G=1, g=0):
    return engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                            engine.mods_from_synth(w.mods), w.max_mods, merge_tol=merge_tol,
                            n_shards=G, shard=g).upload()


@pytest.fixture(scope="module")
def open_parts():
    """Open search (+-500 Da) on a 2000-protein proteome with the medium
    workload's modifications: the whole index and its 2- and 3-way partitions,
    merged lists; plus the oracle's whole-database results."""
    w = synth.workload("medium")
    prot = synth.make_proteome(2000, seed=0)
    sp = w.spectra(prot, n=96, seed=6)
    T = w.frag_tol_bins
    whole = _index(prot, w, T)
    parts = {G: [_index(prot, w, T, G, g) for g in range(G)] for G in (2, 3)}
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                         oracle.mods_from_synth(w.mods), w.max_mods)
    expect = db.search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
    return w, prot, sp, whole, parts, db, expect


def _params(w, schedule=capi.PS_SCHED_PLAIN, **kw):
    a = dict(top_k=w.top_k, min_shared=w.min_shared, max_charge=3, schedule=schedule)
    a.update(kw)
    return engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, **a)


@pytest.mark.parametrize("G", [2, 3])
@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_partitioned_search_assembles_to_whole(open_parts, G, schedule):
    w, prot, sp, whole, parts, db, (oh, ost, og) = open_parts
    _say(f"partitions: G={G} schedule={schedule}, {sp.n} spectra")
    prm = _params(w, schedule)
    ref = engine.search(whole, sp, prm)
    res = engine.search_partitioned(parts[G], sp, prm)
    assert (ost["status"] == 0).sum() > 40
    _assert_identical(res, ref)
    assert_parity(res, oh, ost, og)
    assert res.postings == ref.postings == int(ost["pairs_total"].sum())


def test_partitioned_classic_index_and_other_parameters(open_parts):
    """Four partitions of a classic (unmerged) index, with top_k 16, k_min 2 and
    a narrower window than the fixture's."""
    w, prot, sp, whole, parts, db, _ = open_parts
    _say("partitions: G=4, classic index")
    idx = [engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                            engine.mods_from_synth(w.mods), w.max_mods, n_shards=4, shard=g).upload()
           for g in range(4)]
    prm = engine.search_params(False, 150_000_000, w.frag_tol_bins, w.top_peaks, 16, 2, max_charge=3)
    res = engine.search_partitioned(idx, sp, prm)
    oh, ost, og = db.search(sp, False, 150_000_000, w.frag_tol_bins, w.top_peaks, 16, 2)
    assert_parity(res, oh, ost, og)
    assert _same(res.hits, engine.search(whole, sp, prm).hits)


def test_more_partitions_than_entries():
    """64 partitions of a database with fewer entries: most partitions are empty
    and some spectra score nothing anywhere; also an empty batch."""
    prot = synth.Proteome(np.frombuffer(b"MSTKPEPTIDERAAGLKWWSTYPEPKR", np.uint8).copy(),
                          np.array([0, 27], np.uint64))
    db = oracle.Database(prot.residues, prot.offsets, 2, 3, 20, [], 0)
    n_pep = len(db)
    assert n_pep < 64
    idx = [engine.HostIndex(prot.residues, prot.offsets, 2, 3, 20, [], 0, n_shards=64, shard=g).upload()
           for g in range(64)]
    assert sum(len(i) for i in idx) == n_pep
    peaks, prec = [], []
    for pid in range(n_pep):
        b, y = oracle.ions(db.residue_masses(pid))
        peaks.append([(float(m) * 1e-6, 1.0 + k % 5) for k, m in enumerate(np.concatenate([b, y]))])
        prec.append((db.get(pid)[0] + 2 * 1007276) * 1e-6 / 2)
    peaks.append([(333.0, 1.0)]); prec.append(2000.0)          # matches nothing
    off = np.zeros(len(peaks) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in peaks])
    sp = synth.Spectra(off, np.array([m for p in peaks for m, _ in p], np.float32),
                       np.array([i for p in peaks for _, i in p], np.float32), np.array(prec, np.float64),
                       np.full(len(peaks), 2, np.int8))
    _say(f"partitions: G=64 over {n_pep} entries")
    prm = engine.search_params(False, 5_000_000_000, 1, 100, 5, 1, max_charge=2)
    res = engine.search_partitioned(idx, sp, prm)
    oh, ost, og = db.search(sp, False, 5_000_000_000, 1, 100, 5, 1)
    assert_parity(res, oh, ost, og)
    assert int(res.stats["status"][-1]) == capi.PS_STATUS_NO_HITS
    empty = sp.subset(np.arange(0, 0))
    r0 = engine.search_partitioned(idx, empty, prm)
    assert r0.hits.shape == (0, 5) and r0.stats.shape == (0,)


def test_assembly_keeps_invalid_spectra_invalid(open_parts):
    """Device-resident inputs with invalid spectra, searched on each partition:
    the assembled status stays INVALID and the other spectra match the whole
    search of the valid ones."""
    import torch
    w, prot, sp, whole, parts, db, _ = open_parts
    sub = sp.subset(np.arange(0, 24))
    charge = sub.charge.copy()
    charge[3] = 0
    prec = sub.precursor_mz.copy()
    prec[9] = np.nan
    t = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in
         (sub.peak_off.astype(np.uint64).view(np.int64), sub.mz, sub.intensity, prec, charge)]
    s = capi.ps_spectra(sub.n, *[x.data_ptr() for x in t])
    prm = _params(w)
    nnz = int(sub.peak_off[-1])
    batches, spaces, pp = [], [], []
    _say("partitions: invalid spectra through ps_search_device")
    try:
        for ix in parts[3]:
            need = C.c_uint64()
            capi.check(capi.ps_workspace_bytes(ix.handle, sub.n, nnz, C.byref(prm), C.byref(need)))
            ws = engine.Workspace()
            d = ws.get(need.value)
            bh = C.c_void_p()
            capi.check(capi.ps_search_device(ix.handle, C.byref(d), C.byref(s), nnz, C.byref(prm), C.byref(bh)))
            batches.append(bh)
            spaces.append(ws)
            pp.append(engine._device_results(bh))
        out = engine.AssembleOut(sub.n, prm.top_k)
        engine.assemble(pp, sub.n, prm.top_k, out, fit=prm.fit)
        torch.cuda.synchronize()
        hits, stats, hist = out.to_host()
    finally:
        for bh in batches:
            capi.ps_batch_free(bh)
    assert stats["status"][3] == capi.PS_STATUS_INVALID and stats["status"][9] == capi.PS_STATUS_INVALID
    assert stats["n_window"][3] == 0 and stats["n_scored"][9] == 0
    assert np.all(hits["id"][[3, 9]] == 0xFFFFFFFF)
    good = np.array([i for i in range(sub.n) if i not in (3, 9)])
    ref = engine.search(whole, sub.subset(good), prm)
    assert _same(hits[good], ref.hits) and _same(stats[good], ref.stats) and _same(hist[good], ref.hist)


def test_assembly_of_graph_plan_results(open_parts):
    """Partition searches run as captured plans (persistent schedule); their
    device results assemble to the whole search, over two different batches."""
    import torch
    w, prot, sp, whole, parts, db, _ = open_parts
    prm = _params(w, capi.PS_SCHED_PERSISTENT)
    nnz = int(sp.peak_off[-1])
    plans = [engine.Plan(ix, prm, sp.n, nnz) for ix in parts[2]]
    for batch in (sp.subset(np.arange(0, 60)), sp.subset(np.arange(40, 96))):
        _say(f"partitions: plans, batch of {batch.n}")
        pp = []
        for p in plans:
            p.run(batch)
            p.results()                                 # waits for the run
            h, st, hg = C.c_void_p(), C.c_void_p(), C.c_void_p()
            capi.check(capi.ps_plan_device_results(p.handle, C.byref(h), C.byref(st), C.byref(hg)))
            pp.append(capi.ps_part(h.value, st.value, hg.value, None))
        out = engine.AssembleOut(batch.n, prm.top_k)
        engine.assemble(pp, batch.n, prm.top_k, out, fit=prm.fit)
        torch.cuda.synchronize()
        hits, stats, hist = out.to_host()
        ref = engine.search(whole, batch, prm)
        assert _same(hits, ref.hits) and _same(stats, ref.stats) and _same(hist, ref.hist)


@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_gumbel_fit_parity_whole_and_partitioned(open_parts, schedule):
    """The log-Weibull (Gumbel) expect value: whole-database search against the
    oracle's, and 3 partitions assembled against the whole search bit for bit."""
    w, prot, sp, whole, parts, db, _ = open_parts
    _say(f"gumbel fit: schedule {schedule}")
    prm = _params(w, schedule, fit=capi.PS_FIT_GUMBEL)
    ref = engine.search(whole, sp, prm)
    oh, ost, og = db.search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                            fit=oracle.FIT_GUMBEL)
    assert (ost["status"] == 0).sum() > 60
    assert_parity(ref, oh, ost, og)
    res = engine.search_partitioned(parts[3], sp, prm)
    _assert_identical(res, ref)


# ---------------------------------------------------------------------------
# sampled partial results (Sampling section; the shift of Superstep 4)
# ---------------------------------------------------------------------------

def _synthetic_histograms(n, seed):
    """Histograms of every shape: narrow, wide, long heads and tails, ties
    among the largest counts, counts past 16 bits, at both ends of the range,
    and empty ones."""
    rng = np.random.default_rng(seed)
    hs = np.zeros((n, capi.PS_HIST_BINS), np.int32)
    for i in range(n):
        kind = i % 6
        if kind == 5:
            continue                                    # empty
        a = int(rng.integers(0, capi.PS_HIST_BINS)) if kind != 4 else int(rng.integers(430, 500))
        b = min(capi.PS_HIST_BINS, a + int(rng.integers(1, [30, 121, 300, 512, 200][kind])))
        hs[i, a:b] = rng.integers(0, [3, 50, 1000, 80000, 9][int(rng.integers(0, 5))], b - a)
        if rng.random() < 0.3:
            hs[i, rng.integers(a, b, 3)] = hs[i].max()
    return hs


@pytest.mark.parametrize("n", [1, 5, 1027])
def test_sampling_matches_oracle_records(n):
    """ps_sample against the oracle's records, byte for byte, on histograms of
    every shape (n ragged against the four spectra a workgroup samples)."""
    import torch
    _say(f"sampling: {n} synthetic histograms")
    hs = _synthetic_histograms(n, seed=n)
    ns = np.random.default_rng(1).integers(0, 1 << 40, n).astype(np.uint64)
    stats = np.zeros(n, capi.STAT_DTYPE)
    stats["n_scored"] = ns
    d_hist = torch.from_numpy(hs).cuda()
    d_stats = torch.from_numpy(stats.view(np.uint8)).cuda()
    part = capi.ps_part(None, d_stats.data_ptr(), d_hist.data_ptr(), None)
    _, rec = engine.sample(part, n)
    torch.cuda.synchronize()
    got = engine.sampled_to_host(rec, n)
    want = oracle.sample(hs, ns)
    assert got.tobytes() == want.tobytes()
    assert (got["flags"] & 1).any() and (got["flags"] & 2).any() if n > 100 else True


def _oracle_sampled_assembly(db, sp, w, G, sampled_parts, fit=oracle.FIT_TAIL):
    parts = [db.shard(G, g).search(sp, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k,
                                   w.min_shared, fit=fit) for g in range(G)]
    recs = [oracle.sample(p[2], p[1]["n_scored"]) for p in parts]
    hists = [oracle.unsample(recs[g]) if g in sampled_parts else parts[g][2] for g in range(G)]
    return recs, oracle.assemble([p[0] for p in parts], [p[1] for p in parts], hists, fit=fit)


class _Res:
    def __init__(self, hits, stats, hist):
        self.hits, self.stats, self.hist = hits, stats, hist


@pytest.mark.parametrize("fit", [capi.PS_FIT_TAIL, capi.PS_FIT_GUMBEL])
@pytest.mark.parametrize("sampled_parts", [(0, 1, 2), (1,)])
def test_sampled_assembly_matches_oracle(open_parts, fit, sampled_parts):
    """Three partitions searched on the GPU, their histograms sampled on the
    device (all, or only partition 1), assembled from the samples: equal to the
    oracle's assembly of its own sampled partition results (records byte for
    byte, hits and histograms exact, expect values 1e-5 relative).  Spectra
    whose samples lost nothing equal the full assembly bit for bit."""
    import torch
    w, prot, sp, whole, parts, db, _ = open_parts
    G = 3
    _say(f"sampled assembly: fit {fit}, sampled partitions {sampled_parts}")
    prm = _params(w, capi.PS_SCHED_PLAIN, fit=fit)
    s, keep = engine._spectra_struct(sp)
    ws = [engine.Workspace() for _ in range(G)]
    batches, pp, recs = [], [], []
    try:
        for g, ix in enumerate(parts[G]):
            need = C.c_uint64()
            nnz = int(sp.peak_off[-1])
            capi.check(capi.ps_workspace_bytes(ix.handle, sp.n, nnz, C.byref(prm), C.byref(need)))
            dev = ws[g].get(need.value)
            bh = C.c_void_p()
            capi.check(capi.ps_search_batch(ix.handle, C.byref(dev), C.byref(s), C.byref(prm), C.byref(bh)))
            batches.append(bh)
            full = engine._device_results(bh)
            if g in sampled_parts:
                part, rec = engine.sample(full, sp.n)
                recs.append((g, rec))
                pp.append(part)
            else:
                pp.append(full)
        for bh in batches:
            engine.collect(bh, sp.n, prm)               # waits for the searches
        out = engine.AssembleOut(sp.n, prm.top_k)
        engine.assemble(pp, sp.n, prm.top_k, out, fit=fit)
        full_out = engine.AssembleOut(sp.n, prm.top_k)
        engine.assemble([engine._device_results(bh) for bh in batches], sp.n, prm.top_k, full_out, fit=fit)
        torch.cuda.synchronize()
        hits, stats, hist = out.to_host()
        fh, fst, fhist = full_out.to_host()
        got_recs = {g: engine.sampled_to_host(r, sp.n) for g, r in recs}
    finally:
        for bh in batches:
            capi.ps_batch_free(bh)
    orecs, (oh, ost, og) = _oracle_sampled_assembly(db, sp, w, G, sampled_parts, fit=fit)
    for g, r in got_recs.items():
        assert r.tobytes() == orecs[g].tobytes(), f"records of partition {g} differ"
    assert_parity(_Res(hits, stats, hist), oh, ost, og)
    lossless = np.all([got_recs[g]["flags"] == 0 for g in got_recs], axis=0)
    assert lossless.sum() > 40
    for f, a, b in (("hits", hits, fh), ("stats", stats, fst), ("hist", hist, fhist)):
        assert a[lossless].tobytes() == b[lossless].tobytes(), f

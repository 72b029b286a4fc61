"""The large open-search workload at full size (needs an MI355X).

20k proteins digested with up to two missed cleavages, Met oxidation and STY
phosphorylation with at most three modified sites per peptide: 40.9M peptides
and 6.8G postings in lists merging the three neighbouring bins (27 GB), past
the 2^32 postings a 32-bit position reaches.  The index is built on the GPU and
searched with the schedules and launch forms the benchmark times; sampled
spectra are compared with the oracle, which digests the same proteome itself
and scores every window candidate by generating its ions.  Spectra: 20-200
peaks (all kept, B = 200), precursor masses lognormal around 1800 Da, so
windows of +-500 Da hold 0.1M-10M candidates; charges 2-3 (and 2-4 for the
serving requests' recipe).
"""
import numpy as np
import pytest

import oracle
from paper_2102_02286_amd import capi, engine, synth
from tests.test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def large():
    w = synth.workload("large")
    prot = w.proteome()
    _say("large: building the merged index on the GPU")
    ix = engine.HostIndex.build_on_device(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                                          engine.mods_from_synth(w.mods), w.max_mods, merge_tol=w.frag_tol_bins)
    n_pep, n_post, n_bins = ix.shape()
    _say(f"large: {n_pep} peptides, {n_post} postings, {n_bins} bins; oracle database")
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                         oracle.mods_from_synth(w.mods), w.max_mods)
    assert len(db) == n_pep
    return w, prot, ix, db


def _sample_parity(w, db, sp, res, idx):
    sub = sp.subset(idx)
    _say(f"large: oracle on {len(idx)} sampled spectra")
    oh, ost, og = db.search(sub, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
    from types import SimpleNamespace
    assert_parity(SimpleNamespace(hits=res.hits[idx], stats=res.stats[idx], hist=res.hist[idx]), oh, ost, og)
    return ost


def test_large_index_passes_32bit_positions(large):
    w, prot, ix, db = large
    n_pep, n_post, n_bins = ix.shape()
    assert n_post > 1 << 32
    grain, nbytes = ix.directory()
    assert grain == 12
    # entries equal the oracle's sorted database at sampled ids
    rng = np.random.default_rng(4)
    ent = ix.entries()
    for i in np.concatenate([rng.integers(0, n_pep, 400), [0, n_pep - 1]]):
        assert tuple(ent[int(i)]) == db.get(int(i))


@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_large_sampled_parity(large, schedule):
    """4000 spectra searched together (every tile path, uneven windows); 40 of
    them checked against the oracle, including the largest and smallest
    windows."""
    w, prot, ix, db = large
    sp = w.spectra(prot, n=4000, seed=31)
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=schedule)
    _say(f"large: searching {sp.n} spectra, schedule {schedule}")
    res = engine.search(ix, sp, prm)
    assert res.overflow_spectra == 0
    nw = res.stats["n_window"].astype(np.int64)
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([rng.choice(sp.n, 36, replace=False), [int(np.argmax(nw)), int(np.argmin(nw))],
                                    np.nonzero(np.diff(sp.peak_off.astype(np.int64)) == 200)[0][:1],
                                    np.nonzero(np.diff(sp.peak_off.astype(np.int64)) <= 25)[0][:1]]))
    ost = _sample_parity(w, db, sp, res, idx)
    assert (ost["status"] == 0).sum() >= 30
    assert nw.max() > 8_000_000 and nw.min() < 2_000_000


def test_large_graph_plan_parity(large):
    """The benchmark's launch form: the whole search captured once as a graph
    and replayed for a batch, both schedules giving the same bits."""
    w, prot, ix, db = large
    sp = w.spectra(prot, n=3000, seed=32)
    nnz = int(sp.peak_off[-1])
    out = {}
    for schedule in (capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT):
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                                   max_charge=3, schedule=schedule)
        plan = engine.Plan(ix, prm, n_cap=sp.n, nnz_cap=nnz)
        _say(f"large: graph plan, schedule {schedule}")
        out[schedule] = plan.search(sp)
        del plan
    a, b = out[capi.PS_SCHED_PLAIN], out[capi.PS_SCHED_PERSISTENT]
    assert a.hits.tobytes() == b.hits.tobytes() and a.stats.tobytes() == b.stats.tobytes()
    assert a.hist.tobytes() == b.hist.tobytes()
    idx = np.random.default_rng(8).choice(sp.n, 16, replace=False)
    _sample_parity(w, db, sp, a, np.sort(idx))


def test_large_charge_4_requests_parity(large):
    """The serving recipe's spectra (precursor charges 2-4, so up to three
    fragment charges and 600 probe slots per spectrum) on the same index."""
    w, prot, ix, db = large
    sp = w.spectra(prot, n=1500, seed=33, charges=(2, 3, 4))
    assert (sp.charge == 4).sum() > 400
    for schedule in (capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT):
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                                   max_charge=4, schedule=schedule)
        _say(f"large, charges 2-4: schedule {schedule}")
        res = engine.search(ix, sp, prm)
        if schedule == capi.PS_SCHED_PLAIN:
            ref = res
            idx = np.sort(np.concatenate([np.nonzero(sp.charge == 4)[0][:14],
                                          np.nonzero(sp.charge != 4)[0][:6]]))
            _sample_parity(w, db, sp, res, idx)
        else:
            assert res.hits.tobytes() == ref.hits.tobytes() and res.stats.tobytes() == ref.stats.tobytes()


def test_medium_merged_full_size_sampled_parity():
    """The medium workload as the previous benchmark configuration ran it:
    merged lists (T = 1) built on the host, the full 100k-spectrum batch in one
    graph plan, 24 sampled spectra against the oracle."""
    w = synth.workload("medium")
    prot = w.proteome()
    _say("medium merged: building index")
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(w.mods), w.max_mods, merge_tol=w.frag_tol_bins).upload()
    sp = w.spectra(prot)
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=capi.PS_SCHED_PLAIN)
    plan = engine.Plan(ix, prm, n_cap=sp.n, nnz_cap=int(sp.peak_off[-1]))
    _say(f"medium merged: graph plan over {sp.n} spectra")
    res = plan.search(sp)
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                         oracle.mods_from_synth(w.mods), w.max_mods)
    idx = np.sort(np.random.default_rng(124).choice(sp.n, 24, replace=False))
    _sample_parity(w, db, sp, res, idx)

"""Serving loop on the GPU: continuous batching over a resident index.

Every request's results in the mix must equal the same request searched alone
(bit-exact), whatever it was packed with and whichever slot ran it.
"""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2102_02286_amd import capi, engine, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def served():
    w = synth.workload("medium")
    prot = synth.make_proteome(2000, seed=0)
    sp = w.spectra(prot, n=600, seed=8)
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(w.mods), w.max_mods).upload()
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=capi.PS_SCHED_PERSISTENT)
    return w, prot, sp, ix, prm


def _requests(sp, rng, count, lo=1, hi=60):
    out, at = [], 0
    for _ in range(count):
        k = int(rng.integers(lo, hi + 1))
        idx = (np.arange(at, at + k) % sp.n)
        at += k
        out.append(sp.subset(idx))
    return out


def test_mix_equals_alone(served):
    w, prot, sp, ix, prm = served
    rng = np.random.default_rng(3)
    reqs = _requests(sp, rng, 40)
    srv = engine.Server(ix, prm, slot_spectra=128, slot_peaks=128 * 200, pool_bytes=1 << 30, max_slots=3)
    assert srv.stats().slots == 3
    tickets = [None] * len(reqs)

    def producer():
        for i, r in enumerate(reqs):
            tickets[i] = srv.submit(r)
            time.sleep(float(rng.exponential(0.002)))

    th = threading.Thread(target=producer)
    _say("serving: 40 requests through 3 slots")
    th.start()
    th.join()
    results = [srv.wait(t, r.n) for t, r in zip(tickets, reqs)]
    st = srv.stats()
    srv.close()
    assert st.completed == len(reqs)
    assert st.spectra == sum(r.n for r in reqs)
    assert st.runs <= len(reqs)
    assert 0 < st.p50_ms <= st.p99_ms <= st.max_ms
    for r, (hits, stats, hist, lat) in zip(reqs, results):
        alone = engine.search(ix, r, prm)
        assert hits.tobytes() == alone.hits.tobytes()
        assert stats.tobytes() == alone.stats.tobytes()
        assert hist.tobytes() == alone.hist.tobytes()
        assert lat > 0


def test_mix_matches_oracle(served):
    w, prot, sp, ix, prm = served
    rng = np.random.default_rng(5)
    reqs = _requests(sp, rng, 12, 1, 12)
    srv = engine.Server(ix, prm, slot_spectra=32, slot_peaks=32 * 200, pool_bytes=1 << 29, max_slots=2)
    tickets = [srv.submit(r) for r in reqs]
    _say("serving: 12 requests vs the oracle")
    results = [srv.wait(t, r.n) for t, r in zip(tickets, reqs)]
    srv.close()
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                         oracle.mods_from_synth(w.mods), w.max_mods)
    for r, (hits, stats, hist, lat) in zip(reqs, results):
        oh, ost, og = db.search(r, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
        assert np.array_equal(hits["id"], oh["id"])
        assert np.array_equal(hits["n_b"], oh["n_b"]) and np.array_equal(hits["n_y"], oh["n_y"])
        assert np.array_equal(stats["n_scored"], ost["n_scored"]) and np.array_equal(hist, og)


def test_queue_refusal_and_retry(served):
    """A tiny queue refuses submissions with PS_EAGAIN; retried requests still
    come back identical to searching them alone."""
    w, prot, sp, ix, prm = served
    rng = np.random.default_rng(9)
    reqs = _requests(sp, rng, 16, 20, 40)
    srv = engine.Server(ix, prm, slot_spectra=64, slot_peaks=64 * 200, pool_bytes=1 << 29, max_slots=1,
                        max_pending=1)
    tickets, refused = [], 0
    _say("serving: queue of one")
    for r in reqs:
        while True:
            try:
                tickets.append(srv.submit(r))
                break
            except capi.PsError as e:
                assert e.code == capi.PS_EAGAIN
                refused += 1
                time.sleep(0.001)
    results = [srv.wait(t, r.n) for t, r in zip(tickets, reqs)]
    st = srv.stats()
    srv.close()
    assert refused > 0 and st.refused == refused
    for r, (hits, stats, hist, lat) in zip(reqs, results):
        alone = engine.search(ix, r, prm)
        assert hits.tobytes() == alone.hits.tobytes() and stats.tobytes() == alone.stats.tobytes()


def test_oversized_request_is_rejected(served):
    w, prot, sp, ix, prm = served
    srv = engine.Server(ix, prm, slot_spectra=8, slot_peaks=8 * 200, pool_bytes=1 << 28, max_slots=1)
    with pytest.raises(capi.PsError) as e:
        srv.submit(sp.subset(np.arange(0, 9)))
    assert e.value.code == capi.PS_EINVAL
    srv.close()

"""Serving loop on the GPU: continuous batching over a resident index, with
admission by device memory.

Every request's results in the mix must equal the same request searched alone
(bit-exact), whatever it was packed with and whichever stream ran it, and must
match the oracle: ids, counts and intensity sums, window sizes and histograms
bit for bit, hyperscores bit for bit, expect values within 1e-5 relative.
"""
import ctypes as C
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


def _need(ix, prm, r):
    """Device bytes of request r searched alone (what the server reserves)."""
    b = C.c_uint64()
    capi.check(capi.ps_workspace_bytes(ix.handle, r.n, int(r.peak_off[-1]), C.byref(prm), C.byref(b)))
    return b.value


def _same_as_alone(ix, prm, reqs, results):
    for r, (hits, stats, hist, lat) in zip(reqs, results):
        alone = engine.search(ix, r, prm)
        assert hits.tobytes() == alone.hits.tobytes()
        assert stats.tobytes() == alone.stats.tobytes()
        assert hist.tobytes() == alone.hist.tobytes()
        assert lat > 0


def test_mix_equals_alone(served):
    w, prot, sp, ix, prm = served
    rng = np.random.default_rng(3)
    reqs = _requests(sp, rng, 40)
    srv = engine.Server(ix, prm, pool_bytes=1 << 30, run_spectra=128, max_runs=3)
    assert srv.stats().streams == 3
    tickets = [None] * len(reqs)

    def producer():
        for i, r in enumerate(reqs):
            tickets[i] = srv.submit(r)
            time.sleep(float(rng.exponential(0.002)))

    th = threading.Thread(target=producer)
    _say("serving: 40 requests over 3 streams")
    th.start()
    th.join()
    results = [srv.wait(t, r.n) for t, r in zip(tickets, reqs)]
    st = srv.stats()
    srv.close()
    assert st.completed == len(reqs) and st.samples == len(reqs)
    assert st.spectra == sum(r.n for r in reqs)
    assert st.runs <= len(reqs)
    assert 0 < st.p50_ms <= st.p99_ms <= st.max_ms
    assert 0 < st.peak_bytes <= st.pool_bytes and st.committed_bytes == 0
    _same_as_alone(ix, prm, reqs, results)


def test_mix_matches_oracle(served):
    w, prot, sp, ix, prm = served
    rng = np.random.default_rng(5)
    reqs = _requests(sp, rng, 12, 1, 12)
    srv = engine.Server(ix, prm, pool_bytes=1 << 29, run_spectra=32, max_runs=2)
    tickets = [srv.submit(r) for r in reqs]
    _say("serving: 12 requests vs the oracle")
    results = [srv.wait(t, r.n) for t, r in zip(tickets, reqs)]
    srv.close()
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                         oracle.mods_from_synth(w.mods), w.max_mods)
    for r, (hits, stats, hist, lat) in zip(reqs, results):
        oh, ost, og = db.search(r, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
        for f in ("id", "n_b", "n_y", "sum_q"):
            assert np.array_equal(hits[f], oh[f]), f
        assert hits["hyperscore"].tobytes() == oh["hyperscore"].tobytes()
        for f in ("n_window", "n_scored", "status"):
            assert np.array_equal(stats[f], ost[f]), f
        ok = ost["status"] == 0
        assert np.all(np.isnan(stats["evalue"][~ok]))
        assert np.allclose(stats["evalue"][ok], ost["evalue"][ok], rtol=1e-5, atol=0)
        assert np.array_equal(hist, og)


def test_memory_guard_refuses_then_retries(served):
    """With room for about two requests' device memory, submissions are refused
    with PS_EAGAIN; retried requests come back identical to searching them
    alone."""
    w, prot, sp, ix, prm = served
    rng = np.random.default_rng(9)
    reqs = _requests(sp, rng, 16, 20, 40)
    biggest = max(_need(ix, prm, r) for r in reqs)
    srv = engine.Server(ix, prm, pool_bytes=1 << 29, run_spectra=64, max_runs=1, max_committed_bytes=2 * biggest)
    tickets, refused = [], 0
    _say("serving: memory guard of two requests")
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
    _same_as_alone(ix, prm, reqs, results)


def test_requests_wait_for_memory(served):
    """A pool that holds about one run at a time: requests queue behind each
    other for memory (none is refused, none is skipped), the reserved bytes
    never pass the pool, and every result equals the request alone."""
    w, prot, sp, ix, prm = served
    rng = np.random.default_rng(11)
    reqs = _requests(sp, rng, 10, 30, 50)
    biggest = max(_need(ix, prm, r) for r in reqs)
    pool = (int(1.5 * biggest) + 255) // 256 * 256
    srv = engine.Server(ix, prm, pool_bytes=pool, run_spectra=4096, max_runs=4, max_committed_bytes=64 * biggest)
    _say("serving: one run's worth of pool for ten requests")
    tickets = [srv.submit(r) for r in reqs]
    results = [srv.wait(t, r.n) for t, r in zip(tickets, reqs)]
    st = srv.stats()
    srv.close()
    assert st.refused == 0 and st.completed == len(reqs)
    assert st.peak_bytes <= st.pool_bytes
    _same_as_alone(ix, prm, reqs, results)


def test_large_request_runs_alone_and_oversize_is_refused(served):
    """A request above the packing target runs by itself; one whose device
    memory exceeds the pool is refused with PS_ENOMEM."""
    w, prot, sp, ix, prm = served
    big = sp.subset(np.arange(0, 300))
    srv = engine.Server(ix, prm, pool_bytes=1 << 29, run_spectra=16, max_runs=2)
    _say("serving: a request larger than the packing target")
    hits, stats, hist, _ = srv.wait(srv.submit(big), big.n)
    alone = engine.search(ix, big, prm)
    assert hits.tobytes() == alone.hits.tobytes() and stats.tobytes() == alone.stats.tobytes()
    srv.close()
    small = engine.Server(ix, prm, pool_bytes=_need(ix, prm, sp.subset(np.arange(0, 8))) + 4096, run_spectra=8,
                          max_runs=1)
    with pytest.raises(capi.PsError) as e:
        small.submit(sp.subset(np.arange(0, 64)))
    assert e.value.code == capi.PS_ENOMEM
    small.close()


def test_second_waiter_on_a_ticket_is_refused(served):
    w, prot, sp, ix, prm = served
    srv = engine.Server(ix, prm, pool_bytes=1 << 28, run_spectra=64, max_runs=1)
    r = sp.subset(np.arange(0, 40))
    t = srv.submit(r)
    first = {}

    def waiter():
        first["res"] = srv.wait(t, r.n)

    th = threading.Thread(target=waiter)
    th.start()
    time.sleep(0.05)
    # the first waiter holds the ticket, or has already consumed it: either way a second wait fails
    with pytest.raises(capi.PsError) as e:
        srv.wait(t, r.n)
    assert e.value.code == capi.PS_EINVAL
    th.join()
    assert first["res"][0].shape == (r.n, prm.top_k)
    srv.close()

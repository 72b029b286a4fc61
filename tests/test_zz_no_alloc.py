"""ps_search_static, the search entry point that allocates nothing (needs an
MI355X): its results must equal ps_search_device's bit for bit, call after
call on the shared static work area, the second call with a smaller batch."""
import ctypes as C

import numpy as np
import pytest

from paper_2102_02286_amd import capi, engine, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def setup():
    w = synth.workload("medium")
    prot = synth.make_proteome(2000, seed=0)
    sp = w.spectra(prot, n=300, seed=41)
    ix = engine.HostIndex(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                          engine.mods_from_synth(w.mods), w.max_mods, merge_tol=w.frag_tol_bins).upload()
    return w, sp, ix


def _device_inputs(sp, torch):
    t = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in
         (sp.peak_off.astype(np.uint64).view(np.int64), sp.mz, sp.intensity, sp.precursor_mz, sp.charge)]
    return t, capi.ps_spectra(sp.n, *[x.data_ptr() for x in t])


def _static(ix, sp, prm, want_hist):
    import torch
    tens, dsp = _device_inputs(sp, torch)
    n, k = sp.n, prm.top_k
    hits = torch.zeros(n * k * capi.HIT_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    stats = torch.zeros(n * capi.STAT_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    hist = torch.zeros(n * capi.PS_HIST_BINS * 4, dtype=torch.uint8, device="cuda:0") if want_hist else None
    stream = torch.cuda.current_stream()
    capi.check(capi.ps_search_static(ix.handle, stream.cuda_stream, C.byref(dsp), int(sp.peak_off[-1]), C.byref(prm),
                                     hits.data_ptr(), stats.data_ptr(), hist.data_ptr() if hist is not None else None),
               "ps_search_static")
    torch.cuda.synchronize()
    h = hits.cpu().numpy().view(capi.HIT_DTYPE).reshape(n, k)
    s = stats.cpu().numpy().view(capi.STAT_DTYPE)
    g = hist.cpu().numpy().view(np.int32).reshape(n, capi.PS_HIST_BINS) if hist is not None else None
    return h, s, g


def _device(ix, sp, prm):
    import torch
    tens, dsp = _device_inputs(sp, torch)
    need = C.c_uint64()
    nnz = int(sp.peak_off[-1])
    capi.check(capi.ps_workspace_bytes(ix.handle, sp.n, nnz, C.byref(prm), C.byref(need)))
    ws = engine.Workspace()
    d = ws.get(need.value)
    b = C.c_void_p()
    capi.check(capi.ps_search_device(ix.handle, C.byref(d), C.byref(dsp), nnz, C.byref(prm), C.byref(b)))
    r = engine.collect(b, sp.n, prm)
    capi.ps_batch_free(b)
    return r


@pytest.mark.parametrize("schedule", [capi.PS_SCHED_PLAIN, capi.PS_SCHED_PERSISTENT])
def test_static_search_equals_device_search(setup, schedule):
    w, sp, ix = setup
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3, schedule=schedule)
    small = sp.subset(np.arange(40, 97))
    charge = small.charge.copy()
    charge[5] = 0                                     # an invalid spectrum, reported per spectrum
    small = synth.Spectra(small.peak_off, small.mz, small.intensity, small.precursor_mz, charge)
    for k, (batch, want_hist) in enumerate([(sp, True), (small, False), (sp.subset(np.arange(0, 9)), True)]):
        _say(f"static search call {k}: {batch.n} spectra, schedule {schedule}, histograms {want_hist}")
        h, s, g = _static(ix, batch, prm, want_hist)
        ref = _device(ix, batch, prm)
        assert h.tobytes() == ref.hits.tobytes()
        assert s.tobytes() == ref.stats.tobytes()
        if want_hist:
            assert g.tobytes() == ref.hist.tobytes()
        assert (s["status"] == 0).sum() >= batch.n // 3
    assert s is not None


def test_static_search_refuses_batches_past_the_area(setup):
    """A batch whose work area exceeds the static one is refused before any
    launch; an empty batch is a no-op."""
    import torch
    w, sp, ix = setup
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=3)
    tens, dsp = _device_inputs(sp, torch)
    big = capi.ps_spectra(2_000_000, dsp.peak_off, dsp.mz, dsp.intensity, dsp.precursor_mz, dsp.charge)
    out = torch.zeros(256, dtype=torch.uint8, device="cuda:0")
    rc = capi.ps_search_static(ix.handle, None, C.byref(big), int(sp.peak_off[-1]), C.byref(prm), out.data_ptr(),
                               out.data_ptr(), None)
    assert rc == capi.PS_ENOMEM and "static" in capi.last_error()
    empty = capi.ps_spectra(0, dsp.peak_off, dsp.mz, dsp.intensity, dsp.precursor_mz, dsp.charge)
    assert capi.ps_search_static(ix.handle, None, C.byref(empty), 0, C.byref(prm), None, None, None) == capi.PS_OK
    assert capi.ps_search_static(ix.handle, None, None, 0, C.byref(prm), None, None, None) == capi.PS_EINVAL

"""Python front end: build an index in device memory and search spectra.

Thin layer over the C ABI (capi.py).  PyTorch only supplies device memory
blocks (uint8 tensors) and HIP streams; the search itself runs in the
library's kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import capi
from .capi import check, ptr


def _torch():
    import torch
    return torch


@dataclass
class Mod:
    residues: str
    delta_uda: int
    nterm: bool = False


def mods_from_synth(mods) -> list[Mod]:
    return [Mod(m.residues, int(round(m.delta_da * 1e6)), m.nterm) for m in mods]


def _db_params(missed, min_len, max_len, mods, max_mods, merge_tol=0, n_shards=1, shard=0, ion_types=0):
    arr = (capi.ps_mod * max(1, len(mods)))()
    keep = []
    for i, m in enumerate(mods):
        b = (m.residues or "").encode()
        keep.append(b)
        arr[i].residues = b
        arr[i].nterm = 1 if m.nterm else 0
        arr[i].delta_udalton = int(m.delta_uda)
    p = capi.ps_db_params(missed, min_len, max_len, len(mods), max_mods, merge_tol, n_shards, shard, ion_types, 0, arr)
    return p, (arr, keep)


def search_params(window_is_ppm: bool, window: int, frag_tol_bins: int, top_peaks: int, top_k: int = 5,
                  min_shared: int = 4, max_charge: int = 8, schedule: int = capi.PS_SCHED_PLAIN,
                  want_hist: bool = True, fit: int = capi.PS_FIT_TAIL, noise_permille: int = 0,
                  intensity: int = capi.PS_INTENSITY_LINEAR) -> capi.ps_search_params:
    return capi.ps_search_params(int(window_is_ppm), int(frag_tol_bins), int(window), int(top_peaks), int(top_k),
                                 int(min_shared), int(max_charge), int(schedule), int(bool(want_hist)), int(fit),
                                 int(noise_permille), int(intensity), 0)


class HostIndex:
    """The index built on the host (no GPU needed)."""

    def __init__(self, residues: np.ndarray, offsets: np.ndarray, missed: int, min_len: int, max_len: int,
                 mods: list, max_mods: int, merge_tol: int = 0, n_shards: int = 1, shard: int = 0,
                 ion_types: int = 0):
        """merge_tol = T >= 1 stores, for each bin, the postings of bins b-T..b+T
        (searches must then use frag_tol_bins == T).  n_shards = G > 1 keeps only
        partition `shard` of the sorted database (ranks r with r % G == shard).
        ion_types: PS_ION_* bits of the indexed fragment series (0: b and y)."""
        self._res = np.ascontiguousarray(residues, dtype=np.uint8)
        self._off = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.merge_tol = int(merge_tol)
        self.n_shards, self.shard = int(n_shards), int(shard)
        p, self._keep = _db_params(missed, min_len, max_len, list(mods), max_mods, self.merge_tol, self.n_shards,
                                   self.shard, int(ion_types))
        h = C.c_void_p()
        check(capi.ps_index_create(C.byref(p), ptr(self._res), ptr(self._off), self._off.shape[0] - 1,
                                   C.byref(h)), "ps_index_create")
        self.handle = h
        self.arena = None

    @classmethod
    def build_on_device(cls, residues: np.ndarray, offsets: np.ndarray, missed: int, min_len: int, max_len: int,
                        mods: list, max_mods: int, merge_tol: int = 0, n_shards: int = 1, shard: int = 0,
                        device: str = "cuda:0", stream=None, chunk_pairs: int = 0,
                        ion_types: int = 0) -> "HostIndex":
        """The same index built on the GPU (ps_index_build_device), already resident:
        no upload() needed.  The build's scratch block is freed on return;
        chunk_pairs caps the (bin, posting) pairs sorted at a time (0: default)."""
        torch = _torch()
        self = cls.__new__(cls)
        self._res = np.ascontiguousarray(residues, dtype=np.uint8)
        self._off = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.merge_tol = int(merge_tol)
        self.n_shards, self.shard = int(n_shards), int(shard)
        p, self._keep = _db_params(missed, min_len, max_len, list(mods), max_mods, self.merge_tol, self.n_shards,
                                   self.shard, int(ion_types))
        ib, sb = C.c_uint64(), C.c_uint64()
        n_prot = self._off.shape[0] - 1
        check(capi.ps_index_build_device_bytes(C.byref(p), ptr(self._res), ptr(self._off), n_prot, int(chunk_pairs),
                                               C.byref(ib), C.byref(sb)), "ps_index_build_device_bytes")
        self.arena = torch.empty(max(ib.value, 256), dtype=torch.uint8, device=device)
        scratch = torch.empty(max(sb.value, 256), dtype=torch.uint8, device=device)
        st = stream if stream is not None else torch.cuda.current_stream(self.arena.device)
        dev = capi.ps_device(self.arena.data_ptr(), self.arena.numel(), st.cuda_stream)
        scr = capi.ps_device(scratch.data_ptr(), scratch.numel(), st.cuda_stream)
        h = C.c_void_p()
        self.handle = None
        check(capi.ps_index_build_device(C.byref(p), ptr(self._res), ptr(self._off), n_prot, int(chunk_pairs),
                                         C.byref(dev), C.byref(scr), C.byref(h)), "ps_index_build_device")
        self.handle = h
        del scratch
        return self

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and capi is not None:   # module globals are gone at interpreter exit
            try:
                capi.ps_index_free(h)
            except (AttributeError, TypeError):
                return
            self.handle = None

    def shape(self):
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        check(capi.ps_index_shape(self.handle, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def __len__(self):
        return self.shape()[0]

    def entry(self, pid: int):
        m, p, s, n, k = C.c_int64(), C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint64()
        check(capi.ps_index_entry(self.handle, pid, C.byref(m), C.byref(p), C.byref(s), C.byref(n), C.byref(k)))
        return m.value, p.value, s.value, n.value, k.value

    def entries(self):
        """Every entry as a structured array (mass, prot, start, len, mask)."""
        n = len(self)
        out = np.zeros(n, dtype=[("mass", "<i8"), ("prot", "<u4"), ("start", "<u4"), ("len", "<u4"),
                                 ("mask", "<u8")])
        m = np.zeros(n, np.int64); p = np.zeros(n, np.uint32); s = np.zeros(n, np.uint32)
        ln = np.zeros(n, np.uint8); k = np.zeros(n, np.uint64)
        check(capi.ps_index_entries(self.handle, 0, n, ptr(m), ptr(p), ptr(s), ptr(ln), ptr(k)))
        out["mass"], out["prot"], out["start"], out["len"], out["mask"] = m, p, s, ln, k
        return out

    def peptide(self, pid: int) -> str:
        buf = C.create_string_buffer(512)
        check(capi.ps_peptide(self.handle, pid, buf, 512))
        return buf.value.decode()

    def host_arrays(self):
        _, n_post, n_bins = self.shape()
        off = np.zeros(n_bins + 1, np.uint64)
        post = np.zeros(n_post, np.uint32)
        check(capi.ps_index_host_arrays(self.handle, ptr(off), ptr(post)))
        return off, post

    def schedule(self) -> capi.ps_schedule:
        sc = capi.ps_schedule()
        check(capi.ps_index_get_schedule(self.handle, C.byref(sc)))
        return sc

    def set_schedule(self, **fields) -> capi.ps_schedule:
        sc = self.schedule()
        for k, v in fields.items():
            setattr(sc, k, int(v))
        check(capi.ps_index_set_schedule(self.handle, C.byref(sc)), "ps_index_set_schedule")
        return sc

    def directory(self):
        """(grain_shift, device bytes) of the tile directory."""
        g, b = C.c_uint32(), C.c_uint64()
        check(capi.ps_index_directory(self.handle, C.byref(g), C.byref(b), None))
        return g.value, b.value

    def dense(self):
        """(bins with a dense map, whether searches read them)."""
        n, on = C.c_uint32(), C.c_int()
        bins = np.zeros(capi.PS_MAX_DENSE, np.uint32)
        check(capi.ps_index_dense(self.handle, C.byref(n), ptr(bins), C.byref(on)))
        return bins[:n.value].copy(), bool(on.value)

    def set_dense(self, enabled: bool):
        check(capi.ps_index_set_dense(self.handle, 1 if enabled else 0), "ps_index_set_dense")

    def directory_array(self) -> np.ndarray:
        """Host copy of the tile directory, [n_bins, stride] with stride =
        (n_pep >> grain) + 2 rounded up to a multiple of 4."""
        g, nbytes = self.directory()
        n_pep, _, n_bins = self.shape()
        d = np.zeros(nbytes // 4, np.uint32)
        check(capi.ps_index_directory(self.handle, None, None, ptr(d)))
        return d.reshape(n_bins, ((n_pep >> g) + 2 + 3) // 4 * 4)

    def device_bytes(self) -> int:
        b = C.c_uint64()
        check(capi.ps_index_device_bytes(self.handle, C.byref(b)))
        return b.value

    def upload(self, device: str = "cuda:0", stream=None):
        torch = _torch()
        nbytes = self.device_bytes()
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        st = stream if stream is not None else torch.cuda.current_stream(self.arena.device)
        dev = capi.ps_device(self.arena.data_ptr(), nbytes, st.cuda_stream)
        check(capi.ps_index_upload(self.handle, C.byref(dev)), "ps_index_upload")
        return self


def _spectra_struct(sp):
    arrs = [np.ascontiguousarray(sp.peak_off, np.uint64), np.ascontiguousarray(sp.mz, np.float32),
            np.ascontiguousarray(sp.intensity, np.float32), np.ascontiguousarray(sp.precursor_mz, np.float64),
            np.ascontiguousarray(sp.charge, np.int8)]
    s = capi.ps_spectra(sp.n, *[a.ctypes.data for a in arrs])
    return s, arrs


class Workspace:
    """A reusable device block for batches (grown on demand)."""

    def __init__(self, device: str = "cuda:0", stream=None):
        self.device = device
        self.stream = stream
        self.buf = None

    def get(self, nbytes: int):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=self.device)
        st = self.stream if self.stream is not None else torch.cuda.current_stream(self.buf.device)
        return capi.ps_device(self.buf.data_ptr(), self.buf.numel(), st.cuda_stream)


@dataclass
class Results:
    hits: np.ndarray       # [n, top_k] HIT_DTYPE
    stats: np.ndarray      # [n] STAT_DTYPE
    hist: np.ndarray | None
    scan_ms: float
    postings: int
    lookups: int
    wide_spectra: int = 0
    overflow_spectra: int = 0
    dense_postings: int = 0  # of `postings`, those counted through dense maps
    dense_reads: int = 0     # dense-map reads (candidates times dense probes)


def search(index: HostIndex, sp, params: capi.ps_search_params, ws: Workspace | None = None) -> Results:
    """Search host spectra; blocks until results are back on the host."""
    ws = ws or Workspace()
    s, keep = _spectra_struct(sp)
    need = C.c_uint64()
    nnz = int(sp.peak_off[-1]) if sp.n else 0
    check(capi.ps_workspace_bytes(index.handle, sp.n, nnz, C.byref(params), C.byref(need)), "ps_workspace_bytes")
    dev = ws.get(need.value)
    b = C.c_void_p()
    check(capi.ps_search_batch(index.handle, C.byref(dev), C.byref(s), C.byref(params), C.byref(b)),
          "ps_search_batch")
    try:
        return collect(b, sp.n, params)
    finally:
        capi.ps_batch_free(b)


def autotune(index: HostIndex, sample, params: capi.ps_search_params, cache_path: str | None = None,
             ws: Workspace | None = None, headroom: int = 4):
    """Measure candidate schedules on `sample` and set the fastest on the index.
    Returns (best schedule, list of (schedule dict, scan_ms))."""
    ws = ws or Workspace()
    s, keep = _spectra_struct(sample)
    need = C.c_uint64()
    nnz = int(sample.peak_off[-1]) if sample.n else 0
    check(capi.ps_workspace_bytes(index.handle, sample.n, nnz, C.byref(params), C.byref(need)))
    dev = ws.get(need.value * headroom)
    trials = (capi.ps_tune_trial * 256)()
    nt = C.c_uint32()
    best = capi.ps_schedule()
    check(capi.ps_autotune(index.handle, C.byref(dev), C.byref(s), C.byref(params),
                           cache_path.encode() if cache_path else None, trials, 256, C.byref(nt), C.byref(best)),
          "ps_autotune")
    out = []
    for i in range(min(nt.value, 256)):
        t = trials[i]
        out.append(({f: getattr(t.schedule, f) for f, _ in capi.ps_schedule._fields_ if f != "pad"}, t.scan_ms))
    return best, out


def collect(batch, n: int, params: capi.ps_search_params) -> Results:
    hits = np.zeros(n * params.top_k, capi.HIT_DTYPE)
    stats = np.zeros(n, capi.STAT_DTYPE)
    hist = np.zeros(n * capi.PS_HIST_BINS, np.int32) if params.want_hist else None
    rc = capi.ps_results(batch, ptr(hits), ptr(stats), ptr(hist) if hist is not None else None)
    if rc not in (capi.PS_OK, capi.PS_EOVERFLOW):
        check(rc, "ps_results")
    ms, la, po, lk = C.c_double(), C.c_uint32(), C.c_uint64(), C.c_uint64()
    check(capi.ps_batch_timing(batch, C.byref(ms), C.byref(la), C.byref(po), C.byref(lk)), "ps_batch_timing")
    ct = capi.ps_counters()
    check(capi.ps_batch_counters(batch, C.byref(ct)), "ps_batch_counters")
    return Results(hits.reshape(n, params.top_k), stats,
                   hist.reshape(n, capi.PS_HIST_BINS) if hist is not None else None, ms.value, po.value, lk.value,
                   ct.wide_spectra, ct.overflow_spectra, ct.dense_postings, ct.dense_reads)


def _device_results(batch):
    h, st, hg = C.c_void_p(), C.c_void_p(), C.c_void_p()
    check(capi.ps_batch_device_results(batch, C.byref(h), C.byref(st), C.byref(hg)), "ps_batch_device_results")
    return capi.ps_part(h.value, st.value, hg.value, None)


class AssembleOut:
    """Device buffers for assembled results of n spectra (one block, three regions)."""

    def __init__(self, n: int, top_k: int, device: str = "cuda:0"):
        torch = _torch()
        self.n, self.k = n, top_k
        a = lambda b: (b + 255) // 256 * 256
        self.o_stats = a(n * top_k * capi.HIT_DTYPE.itemsize)
        self.o_hist = self.o_stats + a(n * capi.STAT_DTYPE.itemsize)
        self.buf = torch.empty(max(self.o_hist + n * capi.PS_HIST_BINS * 4, 256), dtype=torch.uint8, device=device)

    def pointers(self):
        b = self.buf.data_ptr()
        return b, b + self.o_stats, b + self.o_hist

    def to_host(self):
        n, k = self.n, self.k
        raw = self.buf.cpu().numpy()
        hits = raw[:n * k * 24].view(capi.HIT_DTYPE).reshape(n, k).copy()
        stats = raw[self.o_stats:self.o_stats + n * 32].view(capi.STAT_DTYPE).copy()
        hist = raw[self.o_hist:self.o_hist + n * capi.PS_HIST_BINS * 4].view(np.int32).reshape(n, capi.PS_HIST_BINS).copy()
        return hits, stats, hist


def sample(part, n: int, stream=None, device: str = "cuda:0", rec=None):
    """Enqueue ps_sample on a partition result `part` (ps_part with full
    histograms).  Returns (the ps_part that gives the 256-byte records instead
    of the histograms, the device tensor holding the records; `rec` reuses one
    of at least n * 256 bytes)."""
    torch = _torch()
    if rec is None:
        rec = torch.empty(max(n, 1) * capi.SAMPLED_DTYPE.itemsize, dtype=torch.uint8, device=device)
    elif rec.numel() < n * capi.SAMPLED_DTYPE.itemsize:
        raise ValueError("record buffer too small")
    st = stream if stream is not None else torch.cuda.current_stream(rec.device)
    check(capi.ps_sample(st.cuda_stream, n, part.hist, part.stats, rec.data_ptr()), "ps_sample")
    return capi.ps_part(part.hits, part.stats, None, rec.data_ptr()), rec


def sampled_to_host(rec, n: int) -> np.ndarray:
    return rec.cpu().numpy()[:n * capi.SAMPLED_DTYPE.itemsize].view(capi.SAMPLED_DTYPE).copy()


def assemble(parts, n: int, top_k: int, out: AssembleOut, stream=None, fit: int = capi.PS_FIT_TAIL):
    """Enqueue ps_assemble over the partition results `parts` (ps_part list)."""
    torch = _torch()
    G = len(parts)
    arr = (capi.ps_part * max(1, G))(*parts)
    st = stream if stream is not None else torch.cuda.current_stream(out.buf.device)
    h, s, g = out.pointers()
    check(capi.ps_assemble(st.cuda_stream, G, arr, n, top_k, int(fit), h, s, g), "ps_assemble")


def search_partitioned(indexes: list, sp, params: capi.ps_search_params, device: str = "cuda:0") -> Results:
    """Search each partition index (HostIndex with n_shards = G, shard = g, in
    order g = 0..G-1) on the same stream, then assemble whole-database results
    on the device (ps_assemble); blocks until they are on the host."""
    torch = _torch()
    G = len(indexes)
    for g, ix in enumerate(indexes):
        if ix.n_shards != G or ix.shard != g:
            raise ValueError(f"index {g} is partition {ix.shard} of {ix.n_shards}, expected {g} of {G}")
    s, keep = _spectra_struct(sp)
    nnz = int(sp.peak_off[-1]) if sp.n else 0
    batches, spaces, parts = [], [], []
    try:
        for ix in indexes:
            need = C.c_uint64()
            check(capi.ps_workspace_bytes(ix.handle, sp.n, nnz, C.byref(params), C.byref(need)))
            ws = Workspace(device)
            dev = ws.get(need.value)
            b = C.c_void_p()
            check(capi.ps_search_batch(ix.handle, C.byref(dev), C.byref(s), C.byref(params), C.byref(b)),
                  "ps_search_batch")
            batches.append(b)
            spaces.append(ws)
            parts.append(_device_results(b))
        out = AssembleOut(sp.n, params.top_k, device)
        assemble(parts, sp.n, params.top_k, out, fit=params.fit)
        torch.cuda.current_stream(out.buf.device).synchronize()
        hits, stats, hist = out.to_host()
        scan_ms = postings = lookups = 0
        for b in batches:
            ms, la, po, lk = C.c_double(), C.c_uint32(), C.c_uint64(), C.c_uint64()
            check(capi.ps_batch_timing(b, C.byref(ms), C.byref(la), C.byref(po), C.byref(lk)))
            scan_ms += ms.value; postings += po.value; lookups += lk.value
        return Results(hits, stats, hist, scan_ms, postings, lookups)
    finally:
        for b in batches:
            capi.ps_batch_free(b)


def search_dump(index: HostIndex, sp, params: capi.ps_search_params, cap: int = 1 << 22,
                ws: Workspace | None = None):
    """Every scored candidate of every spectrum, sorted by (spectrum, id)."""
    ws = ws or Workspace()
    s, keep = _spectra_struct(sp)
    need = C.c_uint64()
    nnz = int(sp.peak_off[-1]) if sp.n else 0
    check(capi.ps_workspace_bytes(index.handle, sp.n, nnz, C.byref(params), C.byref(need)))
    dev = ws.get(need.value + cap * 16 + (1 << 16))
    a = np.zeros(cap, np.uint32); b = np.zeros(cap, np.uint32)
    nb = np.zeros(cap, np.uint16); ny = np.zeros(cap, np.uint16); sq = np.zeros(cap, np.uint32)
    cnt = C.c_uint64()
    check(capi.ps_search_dump(index.handle, C.byref(dev), C.byref(s), C.byref(params), cap, ptr(a), ptr(b),
                              ptr(nb), ptr(ny), ptr(sq), C.byref(cnt)), "ps_search_dump")
    m = cnt.value
    order = np.lexsort((b[:m], a[:m]))
    return a[:m][order], b[:m][order], nb[:m][order], ny[:m][order], sq[:m][order]


class Plan:
    """A reusable, graph-captured search plan for batches up to a capacity."""

    def __init__(self, index: HostIndex, params: capi.ps_search_params, n_cap: int, nnz_cap: int,
                 device: str = "cuda:0", stream=None):
        torch = _torch()
        self.index, self.params, self.n_cap, self.nnz_cap = index, params, n_cap, nnz_cap
        need = C.c_uint64()
        check(capi.ps_plan_bytes(index.handle, n_cap, nnz_cap, C.byref(params), C.byref(need)), "ps_plan_bytes")
        self.buf = torch.empty(max(need.value, 256), dtype=torch.uint8, device=device)
        st = None if stream is None else stream.cuda_stream
        dev = capi.ps_device(self.buf.data_ptr(), self.buf.numel(), st)
        h = C.c_void_p()
        check(capi.ps_plan_create(index.handle, C.byref(dev), n_cap, nnz_cap, C.byref(params), C.byref(h)),
              "ps_plan_create")
        self.handle = h
        self.n = 0

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and capi is not None:   # module globals are gone at interpreter exit
            try:
                capi.ps_plan_free(h)
            except (AttributeError, TypeError):
                return
            self.handle = None

    def run(self, sp):
        s, self._keep = _spectra_struct(sp)
        check(capi.ps_plan_run(self.handle, C.byref(s)), "ps_plan_run")
        self.n = sp.n

    def inputs(self) -> capi.ps_spectra:
        d = capi.ps_spectra()
        check(capi.ps_plan_inputs(self.handle, C.byref(d)))
        return d

    def run_device(self, n: int, nnz: int):
        check(capi.ps_plan_run_device(self.handle, n, nnz), "ps_plan_run_device")
        self.n = n

    def results(self) -> Results:
        n, prm = self.n, self.params
        hits = np.zeros(n * prm.top_k, capi.HIT_DTYPE)
        stats = np.zeros(n, capi.STAT_DTYPE)
        hist = np.zeros(n * capi.PS_HIST_BINS, np.int32) if prm.want_hist else None
        rc = capi.ps_plan_results(self.handle, ptr(hits), ptr(stats), ptr(hist) if hist is not None else None)
        if rc not in (capi.PS_OK, capi.PS_EOVERFLOW):
            check(rc, "ps_plan_results")
        g, sc = C.c_double(), C.c_double()
        po, lk, it = C.c_uint64(), C.c_uint64(), C.c_uint64()
        check(capi.ps_plan_timing(self.handle, C.byref(g), C.byref(sc), C.byref(po), C.byref(lk), C.byref(it)))
        ct = capi.ps_counters()
        check(capi.ps_plan_counters(self.handle, C.byref(ct)), "ps_plan_counters")
        r = Results(hits.reshape(n, prm.top_k), stats,
                    hist.reshape(n, capi.PS_HIST_BINS) if hist is not None else None, sc.value, po.value, lk.value,
                    ct.wide_spectra, ct.overflow_spectra, ct.dense_postings, ct.dense_reads)
        r.graph_ms = g.value
        r.items = it.value
        return r

    def search(self, sp) -> Results:
        self.run(sp)
        return self.results()


class Server:
    """Continuous-batching server over a resident index (see ps_server_create)."""

    def __init__(self, index: HostIndex, params: capi.ps_search_params, pool_bytes: int, run_spectra: int = 4096,
                 run_peaks: int | None = None, max_runs: int = 4, max_committed_bytes: int = 0,
                 device: str = "cuda:0"):
        """pool_bytes of device memory are the arena runs reserve their workspace
        from; queued requests are packed into runs of up to run_spectra spectra
        and run_peaks peaks; max_runs runs overlap on their own streams; a
        submission is refused (PS_EAGAIN) while queued plus running requests
        would need more than max_committed_bytes (0: pool_bytes)."""
        torch = _torch()
        self.index, self.params = index, params
        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device=device)
        dev = capi.ps_device(self.pool.data_ptr(), pool_bytes, None)
        h = C.c_void_p()
        run_peaks = run_peaks if run_peaks is not None else run_spectra * capi.PS_MAX_PEAKS_IN
        check(capi.ps_server_create(index.handle, C.byref(dev), C.byref(params), run_spectra, run_peaks,
                                    max_runs, max_committed_bytes, C.byref(h)), "ps_server_create")
        self.handle = h

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            capi.ps_server_free(h)
            self.handle = None

    __del__ = close

    def submit(self, sp) -> int:
        s, keep = _spectra_struct(sp)
        t = C.c_uint64()
        check(capi.ps_server_submit(self.handle, C.byref(s), C.byref(t)), "ps_server_submit")
        return t.value

    def wait(self, ticket: int, n: int):
        k = self.params.top_k
        hits = np.zeros(n * k, capi.HIT_DTYPE)
        stats = np.zeros(n, capi.STAT_DTYPE)
        hist = np.zeros(n * capi.PS_HIST_BINS, np.int32) if self.params.want_hist else None
        lat = C.c_double()
        check(capi.ps_server_wait(self.handle, ticket, ptr(hits), ptr(stats), ptr(hist) if hist is not None else None,
                                  C.byref(lat)), "ps_server_wait")
        return (hits.reshape(n, k), stats, hist.reshape(n, capi.PS_HIST_BINS) if hist is not None else None,
                lat.value)

    def stats(self) -> capi.ps_serve_stats:
        st = capi.ps_serve_stats()
        check(capi.ps_server_stats(self.handle, C.byref(st)))
        return st

    def reset_stats(self):
        check(capi.ps_server_reset_stats(self.handle))

"""Python access to the brute-force CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``.  The product library never imports,
links or calls anything here.

Inputs are the plain arrays of ``paper_2102_02286_amd.synth`` (the one module
both sides share, which holds none of the search arithmetic).  Masses and
windows are integer micro-Dalton; see oracle.h for every reading.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
HIST_BINS = 512


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain C11, fp64, no FP contraction)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fPIC",
               "-shared", "-pthread", os.path.join(_HERE, "oracle.c"), "-o", _SO + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class Params(C.Structure):
    _fields_ = [("window_is_ppm", C.c_int32), ("window", C.c_int64), ("frag_tol_bins", C.c_int32),
                ("top_peaks", C.c_uint32), ("top_k", C.c_uint32), ("min_shared", C.c_uint32),
                ("fit", C.c_int32), ("noise_permille", C.c_uint32), ("intensity", C.c_int32),
                ("ion_types", C.c_uint32)]


FIT_TAIL, FIT_GUMBEL = 0, 1
INTENSITY_LINEAR, INTENSITY_SQRT = 0, 1
ION_A, ION_B, ION_C, ION_X, ION_Y, ION_Z = 1, 2, 4, 8, 16, 32


HIT_DTYPE = np.dtype([("id", "<u4"), ("n_b", "<u2"), ("n_y", "<u2"), ("sum_q", "<u4"),
                      ("pad", "<u4"), ("hyperscore", "<f8")])
STAT_DTYPE = np.dtype([("n_window", "<u8"), ("n_scored", "<u8"), ("evalue", "<f8"),
                       ("status", "<i4"), ("pad", "<i4"), ("lo", "<u8"), ("hi", "<u8"),
                       ("pairs_total", "<u8")])

SAMPLE_BINS, SAMPLE_HEAD = 120, 60
SAMPLED_DTYPE = np.dtype([("lo", "<u2"), ("flags", "<u2"), ("pad", "<u4"), ("n_scored", "<u8"),
                          ("count", "<u2", (SAMPLE_BINS,))])
assert SAMPLED_DTYPE.itemsize == 256

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        L.orc_db_create.restype = P
        L.orc_db_create.argtypes = [P, P, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                    C.c_uint32, P, P, P, C.c_uint32, C.c_int]
        L.orc_db_free.argtypes = [P]
        L.orc_db_size.restype = C.c_uint64
        L.orc_db_size.argtypes = [P]
        L.orc_db_get.argtypes = [P, C.c_uint64, P, P, P, P, P]
        L.orc_db_residue_masses.restype = C.c_uint32
        L.orc_db_residue_masses.argtypes = [P, C.c_uint64, P, C.c_uint32]
        L.orc_ions.argtypes = [P, C.c_uint32, P, P]
        L.orc_search.restype = C.c_int
        L.orc_search.argtypes = [P, C.c_uint64, P, P, P, P, P, C.POINTER(Params), C.c_int, P, P, P]
        L.orc_scored.restype = C.c_int64
        L.orc_scored.argtypes = [P, P, P, P, C.c_double, C.c_int8, C.POINTER(Params), P, P, P, P,
                                 C.c_uint64]
        L.orc_db_shard.restype = P
        L.orc_db_shard.argtypes = [P, C.c_uint32, C.c_uint32]
        L.orc_assemble.restype = C.c_int
        L.orc_assemble.argtypes = [C.c_uint32, C.c_uint64, C.c_uint32, C.c_int32, P, P, P, P, P, P]
        L.orc_hyperscore.restype = C.c_double
        L.orc_hyperscore.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_sg_smooth.argtypes = [P, P]
        L.orc_evalue.restype = C.c_int
        L.orc_evalue.argtypes = [P, C.c_double, C.c_uint64, P, P, P, P]
        L.orc_evalue_gumbel.restype = C.c_int
        L.orc_evalue_gumbel.argtypes = [P, C.c_double, C.c_uint64, P, P, P, P]
        L.orc_sample.argtypes = [P, C.c_uint64, P]
        L.orc_unsample.argtypes = [P, P]
        _lib = L
    return _lib


def host_threads() -> int:
    """Threads the oracle uses by default: the process's CPUs, capped by
    OMP_NUM_THREADS where the environment sets the process's share."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(share)) if share.isdigit() and int(share) > 0 else n)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


RESIDUE_MASK = {chr(c): 1 << (c - ord("A")) for c in range(ord("A"), ord("Z") + 1)}


@dataclass
class ModSpec:
    residues: str
    delta_uda: int
    nterm: bool = False


def mods_from_synth(mods) -> list[ModSpec]:
    """Convert synth.Mod (float Da) to integer uDa (nearest)."""
    return [ModSpec(m.residues, int(round(m.delta_da * 1e6)), m.nterm) for m in mods]


class Database:
    """Every peptide of the digested, modified proteome, sorted by
    (mass, protein, start, length, site mask); id = rank."""

    def __init__(self, residues: np.ndarray, offsets: np.ndarray, missed: int, min_len: int,
                 max_len: int, mods: list[ModSpec], max_mods: int, threads: int | None = None):
        L = lib()
        self._res = np.ascontiguousarray(residues, dtype=np.uint8)
        self._off = np.ascontiguousarray(offsets, dtype=np.uint64)
        masks = np.array([0 if m.nterm else sum(RESIDUE_MASK[c] for c in m.residues) for m in mods] or [0],
                         dtype=np.uint32)
        nterm = np.array([1 if m.nterm else 0 for m in mods] or [0], dtype=np.int32)
        delta = np.array([m.delta_uda for m in mods] or [0], dtype=np.int64)
        self._h = L.orc_db_create(_ptr(self._res), _ptr(self._off), self._off.shape[0] - 1,
                                  missed, min_len, max_len, len(mods), _ptr(masks), _ptr(nterm),
                                  _ptr(delta), max_mods, int(threads or host_threads()))
        if not self._h:
            raise ValueError("oracle rejected the database parameters")

    def shard(self, n_shards: int, shard: int) -> "Database":
        """Partition `shard` of `n_shards`: entries with rank r % G == g, in order."""
        h = lib().orc_db_shard(self._h, int(n_shards), int(shard))
        if not h:
            raise ValueError("invalid shard")
        out = Database.__new__(Database)
        out._res, out._off, out._h = self._res, self._off, h
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_db_free(h)
            self._h = None

    def __len__(self) -> int:
        return int(lib().orc_db_size(self._h))

    def get(self, pid: int) -> tuple:
        m, p, s, n, k = C.c_int64(), C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint64()
        lib().orc_db_get(self._h, pid, C.byref(m), C.byref(p), C.byref(s), C.byref(n), C.byref(k))
        return m.value, p.value, s.value, n.value, k.value

    def table(self) -> np.ndarray:
        out = np.zeros(len(self), dtype=[("mass", "<i8"), ("prot", "<u4"), ("start", "<u4"),
                                         ("len", "<u4"), ("mask", "<u8")])
        for i in range(len(self)):
            out[i] = self.get(i)
        return out

    def residue_masses(self, pid: int) -> np.ndarray:
        buf = np.zeros(64, dtype=np.int64)
        n = lib().orc_db_residue_masses(self._h, pid, _ptr(buf), 64)
        return buf[:n].copy()

    def search(self, sp, window_is_ppm: bool, window: int, frag_tol_bins: int, top_peaks: int,
               top_k: int = 5, min_shared: int = 4, threads: int | None = None, want_hist=True,
               fit: int = FIT_TAIL, noise_permille: int = 0, intensity: int = INTENSITY_LINEAR,
               ion_types: int = 0):
        n = sp.n
        prm = Params(int(window_is_ppm), int(window), int(frag_tol_bins), int(top_peaks), int(top_k),
                     int(min_shared), int(fit), int(noise_permille), int(intensity), int(ion_types))
        hits = np.zeros(n * top_k, dtype=HIT_DTYPE)
        stats = np.zeros(n, dtype=STAT_DTYPE)
        hist = np.zeros(n * HIST_BINS, dtype=np.int32) if want_hist else None
        arrs = [np.ascontiguousarray(sp.peak_off, np.uint64), np.ascontiguousarray(sp.mz, np.float32),
                np.ascontiguousarray(sp.intensity, np.float32), np.ascontiguousarray(sp.precursor_mz, np.float64),
                np.ascontiguousarray(sp.charge, np.int8)]
        rc = lib().orc_search(self._h, n, *[_ptr(a) for a in arrs], C.byref(prm),
                              threads or host_threads(), _ptr(hits), _ptr(stats),
                              _ptr(hist) if hist is not None else None)
        if rc != 0:
            raise ValueError("oracle rejected the spectra or search parameters")
        return hits.reshape(n, top_k), stats, (hist.reshape(n, HIST_BINS) if hist is not None else None)

    def scored(self, sp, s: int, window_is_ppm: bool, window: int, frag_tol_bins: int,
               top_peaks: int, min_shared: int = 4, cap: int = 1 << 22, noise_permille: int = 0,
               intensity: int = INTENSITY_LINEAR, ion_types: int = 0):
        prm = Params(int(window_is_ppm), int(window), int(frag_tol_bins), int(top_peaks), 1,
                     int(min_shared), FIT_TAIL, int(noise_permille), int(intensity), int(ion_types))
        ids = np.zeros(cap, np.uint32); nb = np.zeros(cap, np.uint16)
        ny = np.zeros(cap, np.uint16); sq = np.zeros(cap, np.uint32)
        off2 = np.ascontiguousarray(sp.peak_off[s:s + 2], np.uint64)
        mz = np.ascontiguousarray(sp.mz, np.float32)
        it = np.ascontiguousarray(sp.intensity, np.float32)
        k = lib().orc_scored(self._h, _ptr(off2), _ptr(mz), _ptr(it), float(sp.precursor_mz[s]),
                             int(sp.charge[s]), C.byref(prm), _ptr(ids), _ptr(nb), _ptr(ny), _ptr(sq), cap)
        if k < 0:
            raise ValueError("oracle rejected the spectrum")
        if k > cap:
            raise OverflowError("scored set larger than cap")
        return ids[:k].copy(), nb[:k].copy(), ny[:k].copy(), sq[:k].copy()


def assemble(part_hits, part_stats, part_hist, fit: int = FIT_TAIL):
    """Assemble G partition results (lists indexed by partition g, each as
    returned by Database.search on Database.shard(G, g)) into whole-database
    results: (hits[n, k], stats[n], hist[n, 512])."""
    G = len(part_hits)
    n, k = part_hits[0].shape
    ph = np.ascontiguousarray(np.stack(part_hits), dtype=HIT_DTYPE)
    ps = np.ascontiguousarray(np.stack(part_stats), dtype=STAT_DTYPE)
    pg = np.ascontiguousarray(np.stack(part_hist), dtype=np.int32)
    hits = np.zeros(n * k, HIT_DTYPE)
    stats = np.zeros(n, STAT_DTYPE)
    hist = np.zeros(n * HIST_BINS, np.int32)
    rc = lib().orc_assemble(G, n, k, int(fit), _ptr(ph), _ptr(ps), _ptr(pg), _ptr(hits), _ptr(stats),
                            _ptr(hist))
    if rc != 0:
        raise ValueError("oracle rejected the assembly arguments")
    return hits.reshape(n, k), stats, hist.reshape(n, HIST_BINS)


def sample(hist: np.ndarray, n_scored) -> np.ndarray:
    """Sampled 256-byte records (oracle.h: orc_sample) of histograms [n, 512]
    with their scored-candidate counts [n]."""
    h = np.ascontiguousarray(np.asarray(hist, dtype=np.int32).reshape(-1, HIST_BINS))
    ns = np.asarray(n_scored, dtype=np.uint64).reshape(-1)
    assert ns.shape[0] == h.shape[0]
    out = np.zeros(h.shape[0], SAMPLED_DTYPE)
    for i in range(h.shape[0]):
        lib().orc_sample(_ptr(h[i]), int(ns[i]), _ptr(out[i:i + 1]))
    return out


def unsample(rec: np.ndarray) -> np.ndarray:
    """The histograms [n, 512] the records stand for (the shift of the assembly)."""
    r = np.ascontiguousarray(np.asarray(rec, dtype=SAMPLED_DTYPE).reshape(-1))
    out = np.zeros((r.shape[0], HIST_BINS), np.int32)
    for i in range(r.shape[0]):
        lib().orc_unsample(_ptr(r[i:i + 1]), _ptr(out[i]))
    return out


def ions(residue_uda: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    r = np.ascontiguousarray(residue_uda, dtype=np.int64)
    n = r.shape[0]
    b = np.zeros(max(n - 1, 0), np.int64)
    y = np.zeros(max(n - 1, 0), np.int64)
    lib().orc_ions(_ptr(r), n, _ptr(b), _ptr(y))
    return b, y


def hyperscore(n_b: int, n_y: int, sum_q: int) -> float:
    return float(lib().orc_hyperscore(n_b, n_y, sum_q))


def sg_smooth(hist: np.ndarray) -> np.ndarray:
    h = np.ascontiguousarray(hist, dtype=np.int32)
    assert h.shape == (HIST_BINS,)
    out = np.zeros(HIST_BINS, np.float64)
    lib().orc_sg_smooth(_ptr(h), _ptr(out))
    return out


def evalue_gumbel(hist: np.ndarray, top_h: float, n_scored: int):
    h = np.ascontiguousarray(hist, dtype=np.int32)
    ev, mu, beta = C.c_double(), C.c_double(), C.c_double()
    npts = C.c_int32()
    st = lib().orc_evalue_gumbel(_ptr(h), float(top_h), int(n_scored), C.byref(ev), C.byref(mu), C.byref(beta),
                                 C.byref(npts))
    return st, ev.value, mu.value, beta.value, npts.value


def evalue(hist: np.ndarray, top_h: float, n_scored: int):
    h = np.ascontiguousarray(hist, dtype=np.int32)
    ev, w, b = C.c_double(), C.c_double(), C.c_double()
    npts = C.c_int32()
    st = lib().orc_evalue(_ptr(h), float(top_h), int(n_scored), C.byref(ev), C.byref(w), C.byref(b),
                          C.byref(npts))
    return st, ev.value, w.value, b.value, npts.value

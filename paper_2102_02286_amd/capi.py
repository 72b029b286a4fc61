"""ctypes binding of libpepscan.so: the C ABI of include/pepscan.h, same names.

Argument marshalling only.  Every step of the search runs in the library's
HIP kernels; this module never computes results itself and raises if the
library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpepscan.so")

PS_OK, PS_EINVAL, PS_ENOMEM, PS_EAGAIN, PS_EDEVICE, PS_EOVERFLOW = 0, 1, 2, 3, 4, 5
PS_STATUS_OK, PS_STATUS_NO_HITS, PS_STATUS_FEW_POINTS, PS_STATUS_BAD_SLOPE, PS_STATUS_INVALID, \
    PS_STATUS_OVERFLOW = 0, 1, 2, 3, 4, 5
PS_HIST_BINS = 512
PS_MAX_DENSE = 8
PS_MAX_PEAKS_IN = 4096
PS_STATIC_SCRATCH_BYTES = 256 << 20
PS_SCHED_PLAIN, PS_SCHED_PERSISTENT = 0, 1
PS_FIT_TAIL, PS_FIT_GUMBEL = 0, 1
PS_INTENSITY_LINEAR, PS_INTENSITY_SQRT = 0, 1

_ERR_NAMES = {1: "PS_EINVAL", 2: "PS_ENOMEM", 3: "PS_EAGAIN", 4: "PS_EDEVICE", 5: "PS_EOVERFLOW"}


class PsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class ps_device(C.Structure):
    _fields_ = [("base", C.c_void_p), ("bytes", C.c_uint64), ("stream", C.c_void_p)]


class ps_mod(C.Structure):
    _fields_ = [("residues", C.c_char_p), ("nterm", C.c_int32), ("pad", C.c_int32),
                ("delta_udalton", C.c_int64)]


class ps_db_params(C.Structure):
    _fields_ = [("missed_cleavages", C.c_uint32), ("min_len", C.c_uint32), ("max_len", C.c_uint32),
                ("n_mods", C.c_uint32), ("max_mods", C.c_uint32), ("merge_tol_bins", C.c_uint32),
                ("n_shards", C.c_uint32), ("shard", C.c_uint32), ("ion_types", C.c_uint32), ("reserved", C.c_uint32),
                ("mods", C.POINTER(ps_mod))]


class ps_spectra(C.Structure):
    _fields_ = [("n", C.c_uint64), ("peak_off", C.c_void_p), ("mz", C.c_void_p), ("intensity", C.c_void_p),
                ("precursor_mz", C.c_void_p), ("charge", C.c_void_p)]


class ps_search_params(C.Structure):
    _fields_ = [("window_is_ppm", C.c_int32), ("frag_tol_bins", C.c_int32), ("window", C.c_int64),
                ("top_peaks", C.c_uint32), ("top_k", C.c_uint32), ("min_shared", C.c_uint32),
                ("max_charge", C.c_uint32), ("schedule", C.c_int32), ("want_hist", C.c_int32),
                ("fit", C.c_int32), ("noise_permille", C.c_uint32), ("intensity", C.c_int32),
                ("reserved", C.c_int32)]


class ps_schedule(C.Structure):
    _fields_ = [("tile", C.c_uint32), ("tiles_per_item", C.c_uint32), ("groups_per_cu", C.c_uint32),
                ("group_threads", C.c_uint32), ("reserved", C.c_uint32 * 2)]


class ps_part(C.Structure):
    _fields_ = [("hits", C.c_void_p), ("stats", C.c_void_p), ("hist", C.c_void_p), ("sampled", C.c_void_p)]


class ps_tune_trial(C.Structure):
    _fields_ = [("schedule", ps_schedule), ("scan_ms", C.c_double), ("same", C.c_int32), ("pad", C.c_int32)]


class ps_counters(C.Structure):
    _fields_ = [("postings", C.c_uint64), ("bin_lookups", C.c_uint64), ("work_items", C.c_uint64),
                ("wide_spectra", C.c_uint64), ("overflow_spectra", C.c_uint64), ("dense_postings", C.c_uint64),
                ("dense_reads", C.c_uint64), ("reserved", C.c_uint64 * 1)]


class ps_serve_stats(C.Structure):
    _fields_ = [("completed", C.c_uint64), ("spectra", C.c_uint64), ("runs", C.c_uint64), ("refused", C.c_uint64),
                ("max_queue", C.c_uint64), ("streams", C.c_uint32), ("pad", C.c_uint32), ("pool_bytes", C.c_uint64),
                ("peak_bytes", C.c_uint64), ("committed_bytes", C.c_uint64), ("samples", C.c_uint64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("max_ms", C.c_double), ("mean_ms", C.c_double),
                ("elapsed_s", C.c_double)]


HIT_DTYPE = np.dtype([("id", "<u4"), ("n_b", "<u2"), ("n_y", "<u2"), ("sum_q", "<u4"), ("pad", "<u4"),
                      ("hyperscore", "<f8")])
STAT_DTYPE = np.dtype([("n_window", "<u8"), ("n_scored", "<u8"), ("evalue", "<f8"), ("status", "<i4"),
                       ("pad", "<i4")])
assert HIT_DTYPE.itemsize == 24 and STAT_DTYPE.itemsize == 32
assert C.sizeof(ps_search_params) == 56
assert C.sizeof(ps_db_params) == 48
PS_ION_A, PS_ION_B, PS_ION_C, PS_ION_X, PS_ION_Y, PS_ION_Z = 1, 2, 4, 8, 16, 32
PS_MAX_SHARDS = 64
PS_SAMPLE_BINS, PS_SAMPLE_HEAD = 120, 60
SAMPLED_DTYPE = np.dtype([("lo", "<u2"), ("flags", "<u2"), ("pad", "<u4"), ("n_scored", "<u8"),
                          ("count", "<u2", (PS_SAMPLE_BINS,))])

_P = C.c_void_p
_U64P = C.POINTER(C.c_uint64)

# (name, restype, argtypes) for every function the header declares
_SIGS = [
    ("ps_last_error", C.c_char_p, []),
    ("ps_index_create", C.c_int, [C.POINTER(ps_db_params), _P, _P, C.c_uint64, C.POINTER(_P)]),
    ("ps_index_device_bytes", C.c_int, [_P, _U64P]),
    ("ps_index_upload", C.c_int, [_P, C.POINTER(ps_device)]),
    ("ps_build_index", C.c_int, [C.POINTER(ps_device), C.POINTER(ps_db_params), _P, _P, C.c_uint64,
                                 C.POINTER(_P)]),
    ("ps_index_shape", C.c_int, [_P, _U64P, _U64P, _U64P]),
    ("ps_index_build_device_bytes", C.c_int, [C.POINTER(ps_db_params), _P, _P, C.c_uint64, C.c_uint64, _U64P,
                                              _U64P]),
    ("ps_index_build_device", C.c_int, [C.POINTER(ps_db_params), _P, _P, C.c_uint64, C.c_uint64,
                                        C.POINTER(ps_device), C.POINTER(ps_device), C.POINTER(_P)]),
    ("ps_index_entry", C.c_int, [_P, C.c_uint64, C.POINTER(C.c_int64), C.POINTER(C.c_uint32),
                                 C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), _U64P]),
    ("ps_index_entries", C.c_int, [_P, C.c_uint64, C.c_uint64, _P, _P, _P, _P, _P]),
    ("ps_peptide", C.c_int, [_P, C.c_uint32, C.c_char_p, C.c_size_t]),
    ("ps_index_host_arrays", C.c_int, [_P, _P, _P]),
    ("ps_index_set_schedule", C.c_int, [_P, C.POINTER(ps_schedule)]),
    ("ps_index_get_schedule", C.c_int, [_P, C.POINTER(ps_schedule)]),
    ("ps_index_directory", C.c_int, [_P, C.POINTER(C.c_uint32), _U64P, C.c_void_p]),
    ("ps_index_dense", C.c_int, [_P, C.POINTER(C.c_uint32), C.c_void_p, C.POINTER(C.c_int)]),
    ("ps_index_set_dense", C.c_int, [_P, C.c_int]),
    ("ps_index_free", None, [_P]),
    ("ps_workspace_bytes", C.c_int, [_P, C.c_uint64, C.c_uint64, C.POINTER(ps_search_params), _U64P]),
    ("ps_search_batch", C.c_int, [_P, C.POINTER(ps_device), C.POINTER(ps_spectra),
                                  C.POINTER(ps_search_params), C.POINTER(_P)]),
    ("ps_search_device", C.c_int, [_P, C.POINTER(ps_device), C.POINTER(ps_spectra), C.c_uint64,
                                   C.POINTER(ps_search_params), C.POINTER(_P)]),
    ("ps_results", C.c_int, [_P, _P, _P, _P]),
    ("ps_search_dump", C.c_int, [_P, C.POINTER(ps_device), C.POINTER(ps_spectra), C.POINTER(ps_search_params),
                                 C.c_uint64, _P, _P, _P, _P, _P, _U64P]),
    ("ps_batch_device_results", C.c_int, [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P)]),
    ("ps_assemble", C.c_int, [_P, C.c_uint32, C.POINTER(ps_part), C.c_uint64, C.c_uint32, C.c_int32, _P, _P, _P]),
    ("ps_sample", C.c_int, [_P, C.c_uint64, _P, _P, _P]),
    ("ps_batch_timing", C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_uint32), _U64P, _U64P]),
    ("ps_batch_counters", C.c_int, [_P, C.POINTER(ps_counters)]),
    ("ps_batch_free", None, [_P]),
    ("ps_search_static", C.c_int, [_P, _P, C.POINTER(ps_spectra), C.c_uint64, C.POINTER(ps_search_params), _P, _P,
                                   _P]),
    ("ps_plan_bytes", C.c_int, [_P, C.c_uint64, C.c_uint64, C.POINTER(ps_search_params), _U64P]),
    ("ps_plan_create", C.c_int, [_P, C.POINTER(ps_device), C.c_uint64, C.c_uint64, C.POINTER(ps_search_params),
                                 C.POINTER(_P)]),
    ("ps_plan_run", C.c_int, [_P, C.POINTER(ps_spectra)]),
    ("ps_plan_inputs", C.c_int, [_P, C.POINTER(ps_spectra)]),
    ("ps_plan_run_device", C.c_int, [_P, C.c_uint64, C.c_uint64]),
    ("ps_plan_results", C.c_int, [_P, _P, _P, _P]),
    ("ps_plan_timing", C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double), _U64P, _U64P, _U64P]),
    ("ps_plan_counters", C.c_int, [_P, C.POINTER(ps_counters)]),
    ("ps_plan_device_results", C.c_int, [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P)]),
    ("ps_plan_stream", C.c_int, [_P, C.POINTER(_P)]),
    ("ps_plan_free", None, [_P]),
    ("ps_autotune", C.c_int, [_P, C.POINTER(ps_device), C.POINTER(ps_spectra), C.POINTER(ps_search_params),
                              C.c_char_p, C.POINTER(ps_tune_trial), C.c_uint32, C.POINTER(C.c_uint32),
                              C.POINTER(ps_schedule)]),
    ("ps_server_create", C.c_int, [_P, C.POINTER(ps_device), C.POINTER(ps_search_params), C.c_uint64, C.c_uint64,
                                   C.c_uint32, C.c_uint64, C.POINTER(_P)]),
    ("ps_server_submit", C.c_int, [_P, C.POINTER(ps_spectra), _U64P]),
    ("ps_server_wait", C.c_int, [_P, C.c_uint64, _P, _P, _P, C.POINTER(C.c_double)]),
    ("ps_server_stats", C.c_int, [_P, C.POINTER(ps_serve_stats)]),
    ("ps_server_reset_stats", C.c_int, [_P]),
    ("ps_server_free", None, [_P]),
]

_lib = None


def lib():
    """The loaded library.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(the search has no CPU fallback)")
        # One HIP runtime per process: torch ships its own libamdhip64.so.7, so it
        # must be loaded first; the library then binds to that runtime by soname
        # instead of pulling a second copy from /opt/rocm.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().ps_last_error().decode(errors="replace")


def check(rc: int, what: str = ""):
    if rc != PS_OK:
        raise PsError(rc, f"{what}: {last_error()}" if what else last_error())
    return rc


def _fn(name):
    def call(*args):
        return getattr(lib(), name)(*args)
    call.__name__ = name
    return call


# raw entry points, same names as the C ABI
ps_last_error = _fn("ps_last_error")
ps_index_create = _fn("ps_index_create")
ps_index_device_bytes = _fn("ps_index_device_bytes")
ps_index_upload = _fn("ps_index_upload")
ps_build_index = _fn("ps_build_index")
ps_index_shape = _fn("ps_index_shape")
ps_index_build_device_bytes = _fn("ps_index_build_device_bytes")
ps_index_build_device = _fn("ps_index_build_device")
ps_index_entry = _fn("ps_index_entry")
ps_index_entries = _fn("ps_index_entries")
ps_peptide = _fn("ps_peptide")
ps_index_host_arrays = _fn("ps_index_host_arrays")
ps_index_set_schedule = _fn("ps_index_set_schedule")
ps_index_get_schedule = _fn("ps_index_get_schedule")
ps_index_directory = _fn("ps_index_directory")
ps_index_dense = _fn("ps_index_dense")
ps_index_set_dense = _fn("ps_index_set_dense")
ps_index_free = _fn("ps_index_free")
ps_workspace_bytes = _fn("ps_workspace_bytes")
ps_search_batch = _fn("ps_search_batch")
ps_search_device = _fn("ps_search_device")
ps_results = _fn("ps_results")
ps_search_dump = _fn("ps_search_dump")
ps_batch_device_results = _fn("ps_batch_device_results")
ps_assemble = _fn("ps_assemble")
ps_sample = _fn("ps_sample")
ps_batch_timing = _fn("ps_batch_timing")
ps_batch_counters = _fn("ps_batch_counters")
ps_batch_free = _fn("ps_batch_free")
ps_search_static = _fn("ps_search_static")
ps_plan_bytes = _fn("ps_plan_bytes")
ps_plan_create = _fn("ps_plan_create")
ps_plan_run = _fn("ps_plan_run")
ps_plan_inputs = _fn("ps_plan_inputs")
ps_plan_run_device = _fn("ps_plan_run_device")
ps_plan_results = _fn("ps_plan_results")
ps_plan_timing = _fn("ps_plan_timing")
ps_plan_counters = _fn("ps_plan_counters")
ps_plan_device_results = _fn("ps_plan_device_results")
ps_plan_stream = _fn("ps_plan_stream")
ps_plan_free = _fn("ps_plan_free")
ps_autotune = _fn("ps_autotune")
ps_server_create = _fn("ps_server_create")
ps_server_submit = _fn("ps_server_submit")
ps_server_wait = _fn("ps_server_wait")
ps_server_stats = _fn("ps_server_stats")
ps_server_reset_stats = _fn("ps_server_reset_stats")
ps_server_free = _fn("ps_server_free")


def ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)

"""ctypes declarations of the C ABI in include/mm.h.

Loads the in-tree libmm_hip.so. If it has not been built yet, it is built
once with hipcc; if that fails, the import fails loudly. There is no other
implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmm_hip.so")
_lib = None
_lock = threading.Lock()

MM_OK = 0
MM_ERR_INVALID_ARG = 1
MM_ERR_INVALID_GRAPH = 2
MM_ERR_OUT_OF_MEMORY = 3
MM_ERR_HIP = 4
MM_ERR_NO_PROGRESS = 5
MM_ERR_UNSUPPORTED = 6
STATUS_NAMES = {
    0: "MM_OK", 1: "MM_ERR_INVALID_ARG", 2: "MM_ERR_INVALID_GRAPH", 3: "MM_ERR_OUT_OF_MEMORY",
    4: "MM_ERR_HIP", 5: "MM_ERR_NO_PROGRESS", 6: "MM_ERR_UNSUPPORTED",
}

MM_OFF_I32, MM_OFF_I64 = 0, 1
MM_LAYOUT_U8, MM_LAYOUT_U32, MM_LAYOUT_U2 = 0, 1, 2
MM_PROTOCOL_CAS, MM_PROTOCOL_TWO_PHASE = 0, 1
MM_VALIDATE, MM_SYMMETRIC, MM_STATS, MM_TIMING, MM_CAPTURE = 1, 2, 4, 8, 16
MM_STATIC_SCRATCH_BYTES = 8 << 20


class mm_tuning(ctypes.Structure):
    _fields_ = [
        ("layout", ctypes.c_int32),
        ("protocol", ctypes.c_int32),
        ("hint", ctypes.c_int32),
        ("wg_size", ctypes.c_int32),
        ("wave_vertices", ctypes.c_int32),
        ("disperse", ctypes.c_int32),
        ("assist_after", ctypes.c_int32),
        ("lazy_init", ctypes.c_int32),
        ("scan_width", ctypes.c_int32),
        ("stream_loads", ctypes.c_int32),
        ("whole_graph_vertices", ctypes.c_int32),
        ("relabel", ctypes.c_int32),
        ("hub_degree", ctypes.c_int32),
        ("hub_chunk", ctypes.c_int32),
        ("whole_graph_lds", ctypes.c_int32),
        ("mesh_wave_vertices", ctypes.c_int32),
        ("wait_release", ctypes.c_int32),
        ("upper_only", ctypes.c_int32),
        ("hub_wave", ctypes.c_int32),
        ("min_waves", ctypes.c_int32),
        ("hot_degree", ctypes.c_int32),
        ("order_lists", ctypes.c_int32),
        ("probe_first", ctypes.c_int32),
        ("occupancy", ctypes.c_int32),
        ("iter_cap", ctypes.c_int64),
    ]


class mm_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "sources", "sources_skipped", "touched", "assist_reads", "reserve_attempts",
        "reserve_conflicts", "reserve_matched", "match_attempts", "match_conflicts",
        "match_matched", "word_retries", "pairs", "loop_trips", "conflict_max")] + [
        ("conflict_hist", ctypes.c_uint64 * 10), ("reserved_", ctypes.c_uint64 * 8)]


class mm_ems_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("touched", ctypes.c_int64),
                ("pairs", ctypes.c_int64), ("reserved_", ctypes.c_int64 * 5)]


def stats_dict(s: mm_stats) -> dict:
    d = {f: int(getattr(s, f)) for f, _ in mm_stats._fields_
         if f not in ("conflict_hist", "reserved_")}
    d["conflict_hist"] = [int(v) for v in s.conflict_hist]
    return d


# Every entry point declared in include/mm.h, with its ctypes signature.
_P, _I32, _I64, _U32, _SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                             ctypes.c_size_t)
SIGNATURES = {
    "mm_default_tuning": (None, [ctypes.POINTER(mm_tuning)]),
    "mm_workspace_bytes": (_SZ, [_I64, ctypes.POINTER(mm_tuning)]),
    "mm_workspace_bytes_graph": (_SZ, [_I64, _I64, ctypes.POINTER(mm_tuning)]),
    "mm_create_device_bytes": (_SZ, [_I64, _I64, ctypes.POINTER(mm_tuning)]),
    "mm_create": (_I32, [_P, _I32, _P, _I64, _I64, _P, _SZ, _U32, ctypes.POINTER(mm_tuning), _P,
                         ctypes.POINTER(_P)]),
    "mm_run": (_I32, [_P, _P, _P]),
    "mm_run_static": (_I32, [_P, _I32, _P, _I64, _I64, _U32, ctypes.POINTER(mm_tuning), _P, _P, _P]),
    "mm_sync": (_I32, [_P, _P]),
    "mm_get_stats": (_I32, [_P, _P, ctypes.POINTER(mm_stats)]),
    "mm_reset_stats": (_I32, [_P, _P]),
    "mm_get_timing": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "mm_destroy": (None, [_P]),
    "mm_batch_workspace_bytes": (_SZ, [_I32, _P, ctypes.POINTER(mm_tuning)]),
    "mm_batch_create_device_bytes": (_SZ, [_I32, _P, _I64, ctypes.POINTER(mm_tuning)]),
    "mm_batch_create": (_I32, [_P, _P, _P, _I32, _I64, _P, _SZ, _U32, ctypes.POINTER(mm_tuning), _P,
                               ctypes.POINTER(_P)]),
    "mm_batch_create_list": (_I32, [_P, _P, _P, _P, _I32, _P, _SZ, _U32, ctypes.POINTER(mm_tuning),
                                    _P, ctypes.POINTER(_P)]),
    "mm_batch_run": (_I32, [_P, _P, _P]),
    "mm_batch_sync": (_I32, [_P, _P]),
    "mm_batch_get_stats": (_I32, [_P, _P, ctypes.POINTER(mm_stats)]),
    "mm_batch_items": (_I64, [_P]),
    "mm_batch_destroy": (None, [_P]),
    "mm_check": (_I32, [_P, _P, _P, ctypes.POINTER(_I64)]),
    "mm_batch_check": (_I32, [_P, _P, _P, ctypes.POINTER(_I64)]),
    "mm_pairs": (_I32, [_P, _P, _P, _P, _I64, ctypes.POINTER(_I64)]),
    "mm_ems_scratch_bytes": (_SZ, [_I64]),
    "mm_ems_run": (_I32, [_P, _P, ctypes.c_uint64, _P, _SZ, _P, ctypes.POINTER(mm_ems_stats)]),
    "mm_probe_ceilings": (_I32, [_I64, _I64, _P, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]),
    "mm_last_error": (ctypes.c_char_p, []),
    "mm_version": (ctypes.c_char_p, []),
}


def load():
    """Returns the loaded library, building it first if it is absent."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build(force=True)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


class MMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status
        self.message = message


def check(status: int) -> None:
    if status != MM_OK:
        msg = load().mm_last_error()
        raise MMError(status, msg.decode() if msg else "")

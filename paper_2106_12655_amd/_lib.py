"""ctypes loader for liblk.so (the C ABI declared in include/lk.h).

Argument marshalling only.  There is no fallback: if the library is missing or
does not load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblk.so")
_lock = threading.Lock()
_lib = None

# lk_status
OK, EINVAL, ENOMEM, EDEVICE, ECAPACITY, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
F32, F64 = 0, 1
PLAIN_F64, MIXED, CROSSINGS, BARNES_HUT = 0, 1, 2, 3
MODES = {"plain": PLAIN_F64, "mixed": MIXED, "crossings": CROSSINGS, "barnes_hut": BARNES_HUT}
FLAG_REFIT, FLAG_AMBIGUOUS, FLAG_NONFINITE, FLAG_BADPAIR, FLAG_BADLOOP = 1, 2, 4, 8, 16
FLAG_SKIPPED = 32
INT_INVALID = -(2 ** 31)
OPT_REFIT_THRESHOLD_PPM, OPT_GRAPH, OPT_TIMING, OPT_TILE_A, OPT_CHUNK_A = 1, 2, 3, 4, 5
OPT_WAVES_PER_CU, OPT_ATAN, OPT_SEGS_PER_LANE, OPT_SEGS_PER_LANE_F64 = 6, 7, 8, 9
OPT_SMALL_BATCH, OPT_CROSSING_TOL, OPT_CROSSING_CULL = 10, 11, 12
OPT_BH_BETA_MILLI, OPT_BH_ORDER, OPT_DZ_MAX_PASSES = 13, 14, 15
OPT_BH_ADAPTIVE, OPT_BH_BETA_MAX_MILLI, OPT_BH_TARGET_PPM = 16, 17, 18
OPT_PAIR_SEARCH = 19
FLAG_INTERSECT = 64
DZ_BSPLINE, DZ_POLYLINE = 0, 1
DZ_KINDS = {"bspline": DZ_BSPLINE, "polyline": DZ_POLYLINE}

EXPORTS = ["lk_create", "lk_destroy", "lk_last_error", "lk_build_pairs", "lk_direct_sum",
           "lk_direct_sum_check", "lk_direct_sum_noalloc", "lk_verify", "lk_set_option",
           "lk_set_view_direction", "lk_get_view_direction", "lk_get_stats", "lk_autotune",
           "lk_reserve", "lk_discretize",
           "lk_server_create", "lk_server_destroy", "lk_server_last_error",
           "lk_server_open_session", "lk_server_close_session", "lk_server_submit",
           "lk_server_wait"]
MEM_HOST, MEM_DEVICE = 0, 1


class Stats(ctypes.Structure):
    _fields_ = [("refits", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("refit_kernel_ms", ctypes.c_double),
                ("timed_calls", ctypes.c_int32), ("graph_replayed", ctypes.c_int32), ("tile_a", ctypes.c_int32),
                ("chunk_a", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("atan_form", ctypes.c_int32), ("segs_per_lane", ctypes.c_int32),
                ("refits_direct_sum", ctypes.c_int64), ("bh_list_peak", ctypes.c_int64),
                ("bh_near_pairs", ctypes.c_int64), ("bh_list_cap", ctypes.c_int64),
                ("bh_reruns", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("segs_per_lane", ctypes.c_int32), ("segs_per_lane_f64", ctypes.c_int32),
                ("tile_a", ctypes.c_int32), ("chunk_a", ctypes.c_int32),
                ("small_batch", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("evaluated", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("atan_form", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("n_pairs", ctypes.c_int64), ("n_mismatch", ctypes.c_int64),
                ("n_flagged", ctypes.c_int64), ("refits", ctypes.c_int64),
                ("terms", ctypes.c_double), ("bytes", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class DzInfo(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("input_spans", ctypes.c_int64), ("vertices", ctypes.c_int64),
                ("splits", ctypes.c_int64), ("unfinished", ctypes.c_int64)]


class LkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("lk status %d: %s" % (status, msg))
        self.status = status


def load():
    """Load liblk.so once; raise if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblk.so is not built (%s); run `python -m "
                               "paper_2106_12655_amd.build`" % LIB_PATH)
        # One HIP runtime per process: torch ships its own libamdhip64 and
        # loads it into the global symbol scope, so importing torch first makes
        # liblk.so's HIP calls bind to that same runtime (device memory and
        # stream handles are then shared objects).  Loading liblk.so first
        # would start a second runtime that torch's cannot coexist with.
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        p, i32, i64, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int
        lib.lk_create.argtypes = [ctypes.POINTER(p), ctypes.c_int]
        lib.lk_create.restype = st
        lib.lk_destroy.argtypes = [p]
        lib.lk_destroy.restype = None
        lib.lk_last_error.argtypes = [p]
        lib.lk_last_error.restype = ctypes.c_char_p
        lib.lk_build_pairs.argtypes = [p, p, ctypes.c_int, p, i32, p, i64,
                                       ctypes.POINTER(ctypes.c_int64), p]
        lib.lk_build_pairs.restype = st
        lib.lk_direct_sum.argtypes = [p, p, ctypes.c_int, p, i32, p, i64, ctypes.c_int, p, p, p, p]
        lib.lk_direct_sum.restype = st
        lib.lk_direct_sum_check.argtypes = [p, p, ctypes.c_int, p, i32, p, i64, p, ctypes.c_int,
                                             ctypes.c_int, p, p, p, p, p]
        lib.lk_direct_sum_check.restype = st
        lib.lk_direct_sum_noalloc.argtypes = [p, p, ctypes.c_int, p, i32, p, i64, ctypes.c_int, p,
                                              p, p, p]
        lib.lk_direct_sum_noalloc.restype = st
        lib.lk_verify.argtypes = [p, p, p, i64, p, p, i64, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int64), p, i64, p]
        lib.lk_verify.restype = st
        lib.lk_set_option.argtypes = [p, ctypes.c_int, i64]
        lib.lk_set_option.restype = st
        lib.lk_set_view_direction.argtypes = [p, ctypes.POINTER(ctypes.c_double)]
        lib.lk_set_view_direction.restype = st
        lib.lk_get_view_direction.argtypes = [p, ctypes.POINTER(ctypes.c_double)]
        lib.lk_get_view_direction.restype = st
        lib.lk_get_stats.argtypes = [p, ctypes.POINTER(Stats)]
        lib.lk_get_stats.restype = st
        lib.lk_autotune.argtypes = [p, p, ctypes.c_int, p, i32, p, i64, ctypes.c_int, p, p, p,
                                    ctypes.c_char_p, ctypes.POINTER(Tuning), p]
        lib.lk_autotune.restype = st
        lib.lk_discretize.argtypes = [p, p, p, i32, ctypes.c_int, p, i64, p, i64, p, p,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(DzInfo), p]
        lib.lk_discretize.restype = st
        lib.lk_reserve.argtypes = [p, i32, i64, i64]
        lib.lk_reserve.restype = st
        lib.lk_server_create.argtypes = [ctypes.POINTER(p), ctypes.c_int, i32, i64, ctypes.c_int,
                                         i32, i64]
        lib.lk_server_create.restype = st
        lib.lk_server_destroy.argtypes = [p]
        lib.lk_server_destroy.restype = None
        lib.lk_server_last_error.argtypes = [p]
        lib.lk_server_last_error.restype = ctypes.c_char_p
        lib.lk_server_open_session.argtypes = [p, p, i32, p, p, i64, ctypes.POINTER(ctypes.c_int64)]
        lib.lk_server_open_session.restype = st
        lib.lk_server_close_session.argtypes = [p, i64]
        lib.lk_server_close_session.restype = st
        lib.lk_server_submit.argtypes = [p, i64, p, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int64)]
        lib.lk_server_submit.restype = st
        lib.lk_server_wait.argtypes = [p, i64, i32, ctypes.POINTER(Result), p, p, p, p, i64]
        lib.lk_server_wait.restype = st
        _lib = lib
        return lib


def check(lib, ctx, status: int) -> int:
    if status != OK:
        msg = lib.lk_last_error(ctx)
        raise LkError(status, msg.decode() if msg else "")
    return status

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
PLAIN_F64, MIXED = 0, 1
FLAG_REFIT, FLAG_AMBIGUOUS, FLAG_NONFINITE, FLAG_BADPAIR, FLAG_BADLOOP = 1, 2, 4, 8, 16
INT_INVALID = -(2 ** 31)
OPT_REFIT_THRESHOLD_PPM, OPT_GRAPH, OPT_TIMING, OPT_TILE_A, OPT_CHUNK_A = 1, 2, 3, 4, 5
OPT_WAVES_PER_CU, OPT_ATAN, OPT_SEGS_PER_LANE, OPT_SEGS_PER_LANE_F64 = 6, 7, 8, 9
OPT_SMALL_BATCH = 10

EXPORTS = ["lk_create", "lk_destroy", "lk_last_error", "lk_build_pairs", "lk_direct_sum",
           "lk_verify", "lk_set_option", "lk_get_stats"]


class Stats(ctypes.Structure):
    _fields_ = [("refits", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("refit_kernel_ms", ctypes.c_double),
                ("timed_calls", ctypes.c_int32), ("graph_replayed", ctypes.c_int32), ("tile_a", ctypes.c_int32),
                ("chunk_a", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("atan_form", ctypes.c_int32), ("segs_per_lane", ctypes.c_int32)]


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
        lib.lk_verify.argtypes = [p, p, p, i64, p, p, i64, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int64), p, i64, p]
        lib.lk_verify.restype = st
        lib.lk_set_option.argtypes = [p, ctypes.c_int, i64]
        lib.lk_set_option.restype = st
        lib.lk_get_stats.argtypes = [p, ctypes.POINTER(Stats)]
        lib.lk_get_stats.restype = st
        _lib = lib
        return lib


def check(lib, ctx, status: int) -> int:
    if status != OK:
        msg = lib.lk_last_error(ctx)
        raise LkError(status, msg.decode() if msg else "")
    return status

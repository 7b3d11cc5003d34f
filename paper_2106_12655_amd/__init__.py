"""MI355X-native direct summation of the Gauss linking integral.

Python face of liblk.so (include/lk.h).  Every step of the computation runs in
the HIP kernels of ``csrc/``; this module only marshals torch tensors (device
memory and the current stream) into the C ABI.  It has no CPU fallback: without
a built library or a GPU every call raises.

Functions follow the paper's pipeline (Qu & James 2021, Alg. 1):
``build_pairs`` (potential link search, Alg. 2), ``discretize`` (curves to
polylines with the same linking numbers, Alg. 3), ``direct_sum`` (stage 3 by
direct summation of Eq. 4, Alg. 5; the modes "crossings" and "barnes_hut" run
Alg. 4 and Alg. 6 instead), ``direct_sum_check`` (the same fused with the
certificate comparison and its early exit, Sec. 3.1) and ``verify`` (the
before/after comparison of two sparse matrices, Sec. 3.1).
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (FLAG_AMBIGUOUS, FLAG_BADLOOP, FLAG_BADPAIR, FLAG_INTERSECT, FLAG_NONFINITE,
                   FLAG_REFIT, FLAG_SKIPPED, INT_INVALID, LkError)

__all__ = ["Context", "build_pairs", "discretize", "direct_sum", "direct_sum_check", "verify",
           "LkError", "FLAG_REFIT", "FLAG_AMBIGUOUS", "FLAG_NONFINITE", "FLAG_BADPAIR",
           "FLAG_BADLOOP", "FLAG_SKIPPED", "FLAG_INTERSECT", "INT_INVALID"]


def _torch():
    import torch
    return torch


def _ptr(t) -> int:
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return _lib.F32
    if t.dtype == torch.float64:
        return _lib.F64
    raise TypeError("xyz must be float32 or float64, got %s" % t.dtype)


class Context:
    """One lk_ctx on a HIP device (workspace, graph cache, options)."""

    def __init__(self, device: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.lib = _lib.load()
        self.device = int(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib, None, self.lib.lk_create(ctypes.byref(h), self.device))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.lk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        return _lib.check(self.lib, self.h, st)

    def _dev(self, t, dtype=None, name="tensor"):
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.device.type != "cuda" or (t.device.index or 0) != self.device:
            raise ValueError("%s must live on cuda:%d" % (name, self.device))
        if dtype is not None and t.dtype != dtype:
            raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        return t

    def set_option(self, key: int, value: int):
        self._check(self.lib.lk_set_option(self.h, int(key), int(value)))

    def set_view_direction(self, direction):
        """Projection direction of mode ``"crossings"`` (lk_set_view_direction)."""
        d = (ctypes.c_double * 3)(*[float(x) for x in direction])
        self._check(self.lib.lk_set_view_direction(self.h, d))

    def view_direction(self) -> tuple:
        """The direction in use: scaled to largest magnitude 1, FP32 values."""
        d = (ctypes.c_double * 3)()
        self._check(self.lib.lk_get_view_direction(self.h, d))
        return tuple(d)

    def stats(self) -> dict:
        s = _lib.Stats()
        self._check(self.lib.lk_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in s._fields_}

    # ------------------------------------------------------------ the calls
    def build_pairs(self, xyz, offsets, capacity: int | None = None):
        """Alg. 2: all i<j with overlapping closed AABBs, as int32 [P, 2] on the device."""
        torch = _torch()
        self._dev(xyz, None, "xyz")
        self._dev(offsets, torch.int64, "offsets")
        L = offsets.numel() - 1
        n = ctypes.c_int64(0)
        # a first guess of 8 pairs per loop; the exact count comes back with
        # LK_ECAPACITY when it is too small, and the search runs again
        cap = int(capacity) if capacity is not None else 8 * max(L, 0) + 1024
        out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=xyz.device)
        st = self.lib.lk_build_pairs(self.h, _ptr(xyz), _dtype_code(xyz), _ptr(offsets), L,
                                     _ptr(out) if cap > 0 else ctypes.c_void_p(0), cap,
                                     ctypes.byref(n), _stream(self.device))
        if st == _lib.ECAPACITY and capacity is None:
            cap = int(n.value)
            out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=xyz.device)
            st = self.lib.lk_build_pairs(self.h, _ptr(xyz), _dtype_code(xyz), _ptr(offsets), L,
                                         _ptr(out), cap, ctypes.byref(n), _stream(self.device))
        self._check(st)
        return out[: int(n.value)]

    def discretize(self, ctrl, offsets, pairs, kind: str = "bspline",
                   capacity: int | None = None):
        """Alg. 3 (lk_discretize): closed curves -> polylines with the same
        linking numbers.  ``ctrl`` float64 [N, 3] (B-spline control points or
        polyline vertices, ``kind``), ``offsets`` int64 [L+1], ``pairs`` int32
        [P, 2], all on the device.  Returns ``(xyz float64 [V, 3], offsets int64
        [L+1], loop_flags int32 [L], info dict)`` on the device."""
        torch = _torch()
        self._dev(ctrl, torch.float64, "ctrl")
        self._dev(offsets, torch.int64, "offsets")
        self._dev(pairs, torch.int32, "pairs")
        if pairs.numel() and (pairs.dim() != 2 or pairs.shape[1] != 2):
            raise ValueError("pairs must be [P, 2]")
        P = pairs.shape[0] if pairs.dim() == 2 else 0
        L = offsets.numel() - 1
        dev = ctrl.device
        cap = int(capacity) if capacity is not None else 4 * (ctrl.numel() // 3) + 1024
        off_out = torch.empty(L + 1, dtype=torch.int64, device=dev)
        flags = torch.empty(max(L, 1), dtype=torch.int32, device=dev)
        n = ctypes.c_int64(0)
        info = _lib.DzInfo()
        for attempt in range(2):
            xyz = torch.empty((max(cap, 1), 3), dtype=torch.float64, device=dev)
            st = self.lib.lk_discretize(self.h, _ptr(ctrl), _ptr(offsets), L,
                                        _lib.DZ_KINDS[kind], _ptr(pairs), P, _ptr(xyz), cap,
                                        _ptr(off_out), _ptr(flags), ctypes.byref(n),
                                        ctypes.byref(info), _stream(self.device))
            if st == _lib.ECAPACITY and capacity is None and attempt == 0:
                cap = int(n.value)
                continue
            break
        self._check(st)
        return (xyz[: int(n.value)], off_out, flags[:L],
                {k: getattr(info, k) for k, _ in info._fields_ if k != "reserved"})

    def direct_sum(self, xyz, offsets, pairs, mode: str = "mixed", out=None):
        """Eq. 4 summed over every segment pair of every loop pair.

        Returns ``(lk_real float64[P], lk_int int32[P], flags int32[P])`` on the
        device.  ``flags`` holds the C call's uint32 LK_FLAG_* words in an
        int32 tensor (torch has few uint32 operations); every defined bit is
        below 2^31, so the values read the same.  ``mode`` is ``"mixed"``
        (FP32 terms, FP64 pair sums and FP64 refit of ambiguous pairs),
        ``"plain"`` (FP64 throughout), ``"crossings"`` (certified crossing
        count of a projection, Alg. 4, with the FP64 direct sum for undecided
        pairs) or ``"barnes_hut"`` (the two-tree method of Alg. 6, with the
        FP64 refit of pairs far from an integer).  ``out``: optional
        preallocated output triple.
        """
        torch = _torch()
        self._dev(xyz, None, "xyz")
        self._dev(offsets, torch.int64, "offsets")
        self._dev(pairs, torch.int32, "pairs")
        P = pairs.shape[0] if pairs.dim() == 2 else 0
        if pairs.numel() and (pairs.dim() != 2 or pairs.shape[1] != 2):
            raise ValueError("pairs must be [P, 2]")
        if out is None:
            real = torch.empty(P, dtype=torch.float64, device=xyz.device)
            lk = torch.empty(P, dtype=torch.int32, device=xyz.device)
            flags = torch.empty(P, dtype=torch.int32, device=xyz.device)
        else:
            real, lk, flags = out
        m = _lib.MODES[mode]
        self._check(self.lib.lk_direct_sum(self.h, _ptr(xyz), _dtype_code(xyz), _ptr(offsets),
                                           offsets.numel() - 1, _ptr(pairs), P, m, _ptr(real),
                                           _ptr(lk), _ptr(flags), _stream(self.device)))
        return real, lk, flags

    def direct_sum_noalloc(self, xyz, offsets, pairs, mode: str = "mixed", out=None):
        """lk_direct_sum_noalloc: as :meth:`direct_sum` in the ``"mixed"`` and
        ``"plain"`` modes, with the workspace in the library's static device
        array (at most 65,536 loops and 131,072 pairs; calls on one device must
        not overlap).  Pass ``out`` to keep this binding from allocating the
        outputs; ``out[2]`` (flags) may be None."""
        torch = _torch()
        self._dev(xyz, None, "xyz")
        self._dev(offsets, torch.int64, "offsets")
        self._dev(pairs, torch.int32, "pairs")
        P = pairs.shape[0] if pairs.dim() == 2 else 0
        if pairs.numel() and (pairs.dim() != 2 or pairs.shape[1] != 2):
            raise ValueError("pairs must be [P, 2]")
        if out is None:
            out = (torch.empty(P, dtype=torch.float64, device=xyz.device),
                   torch.empty(P, dtype=torch.int32, device=xyz.device),
                   torch.empty(P, dtype=torch.int32, device=xyz.device))
        real, lk, flags = out
        self._check(self.lib.lk_direct_sum_noalloc(
            self.h, _ptr(xyz), _dtype_code(xyz), _ptr(offsets), offsets.numel() - 1, _ptr(pairs), P,
            _lib.MODES[mode], _ptr(real), _ptr(lk), _ptr(flags), _stream(self.device)))
        return real, lk, flags

    def direct_sum_check(self, xyz, offsets, pairs, expected, early_exit: bool = False,
                         mode: str = "mixed", out=None):
        """Eq. 4 summed per pair with the fused certificate check
        (lk_direct_sum_check): each pair's integer is compared with
        ``expected`` (int32 [P]) as soon as it is final.  Returns
        ``(lk_real, lk_int, flags, n_mismatch)``, all on the device
        (``n_mismatch``: int64 [1]).  With ``early_exit`` the kernels stop
        after the first mismatch; unfinished pairs carry FLAG_SKIPPED."""
        torch = _torch()
        self._dev(xyz, None, "xyz")
        self._dev(offsets, torch.int64, "offsets")
        self._dev(pairs, torch.int32, "pairs")
        self._dev(expected, torch.int32, "expected")
        P = pairs.shape[0] if pairs.dim() == 2 else 0
        if expected.numel() != P:
            raise ValueError("expected must have one entry per pair")
        if out is None:
            out = (torch.empty(P, dtype=torch.float64, device=xyz.device),
                   torch.empty(P, dtype=torch.int32, device=xyz.device),
                   torch.empty(P, dtype=torch.int32, device=xyz.device),
                   torch.empty(1, dtype=torch.int64, device=xyz.device))
        real, lk, flags, nm = out
        m = _lib.MODES[mode]
        self._check(self.lib.lk_direct_sum_check(
            self.h, _ptr(xyz), _dtype_code(xyz), _ptr(offsets), offsets.numel() - 1, _ptr(pairs), P,
            _ptr(expected), 1 if early_exit else 0, m, _ptr(real), _ptr(lk), _ptr(flags), _ptr(nm),
            _stream(self.device)))
        return real, lk, flags, nm

    def autotune(self, xyz, offsets, pairs, mode: str = "mixed", cache_path: str | None = None,
                 out=None) -> dict:
        """Time kernel configurations on this call and keep the fastest
        (lk_autotune); returns the chosen configuration and its timings."""
        torch = _torch()
        self._dev(xyz, None, "xyz")
        self._dev(offsets, torch.int64, "offsets")
        self._dev(pairs, torch.int32, "pairs")
        P = pairs.shape[0]
        if out is None:
            out = (torch.empty(P, dtype=torch.float64, device=xyz.device),
                   torch.empty(P, dtype=torch.int32, device=xyz.device),
                   torch.empty(P, dtype=torch.int32, device=xyz.device))
        t = _lib.Tuning()
        m = _lib.MODES[mode]
        self._check(self.lib.lk_autotune(self.h, _ptr(xyz), _dtype_code(xyz), _ptr(offsets),
                                         offsets.numel() - 1, _ptr(pairs), P, m, _ptr(out[0]),
                                         _ptr(out[1]), _ptr(out[2]),
                                         cache_path.encode() if cache_path else None,
                                         ctypes.byref(t), _stream(self.device)))
        return {k: getattr(t, k) for k, _ in t._fields_}

    def verify(self, pairs, lk, exp_pairs, exp_lk, early_exit: bool = False, cap: int = 1024):
        """Compare (pairs, lk) with (exp_pairs, exp_lk); returns
        ``(n_mismatch, records int32 [k, 4] on the device)`` with records
        ``(i, j, got, expected)`` in pair order."""
        torch = _torch()
        for t, nme in ((pairs, "pairs"), (lk, "lk"), (exp_pairs, "exp_pairs"), (exp_lk, "exp_lk")):
            self._dev(t, torch.int32, nme)
        n = ctypes.c_int64(0)
        rec = torch.empty((max(cap, 1), 4), dtype=torch.int32, device=lk.device)
        self._check(self.lib.lk_verify(self.h, _ptr(pairs), _ptr(lk), lk.numel(), _ptr(exp_pairs),
                                       _ptr(exp_lk), exp_lk.numel(), 1 if early_exit else 0,
                                       ctypes.byref(n), _ptr(rec) if cap > 0 else ctypes.c_void_p(0),
                                       int(cap), _stream(self.device)))
        k = min(int(n.value), int(cap))
        return int(n.value), rec[:k]


_default: dict[int, Context] = {}


def context(device: int = 0) -> Context:
    """The per-device default context."""
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def build_pairs(xyz, offsets, capacity=None):
    return context(xyz.device.index or 0).build_pairs(xyz, offsets, capacity)


def direct_sum(xyz, offsets, pairs, mode="mixed", out=None):
    return context(xyz.device.index or 0).direct_sum(xyz, offsets, pairs, mode, out)


def direct_sum_check(xyz, offsets, pairs, expected, early_exit=False, mode="mixed", out=None):
    return context(xyz.device.index or 0).direct_sum_check(xyz, offsets, pairs, expected,
                                                           early_exit, mode, out)


def discretize(ctrl, offsets, pairs, kind="bspline", capacity=None):
    return context(ctrl.device.index or 0).discretize(ctrl, offsets, pairs, kind, capacity)


def verify(pairs, lk, exp_pairs, exp_lk, early_exit=False, cap=1024):
    return context(lk.device.index or 0).verify(pairs, lk, exp_pairs, exp_lk, early_exit, cap)

"""Plain FP64 CPU oracle for the direct-summation linking number.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_2106_12655_amd``) and never imports it; the two
meet only through the seeded input generators, which hold none of the method's
arithmetic.

The arithmetic lives in ``lk_oracle.c`` (plain C, double precision, libm
``atan2``/``sqrt``), built with gcc by :func:`build`.  Every routine follows a
passage of Qu & James, "Fast Linking Numbers for Topology Verification of Loopy
Structures" (SIGGRAPH 2021):

* :func:`term` -- Eq. 4 (per segment-pair signed solid angle / 2 pi), as printed.
* :func:`term_midpoint` -- the midpoint quadrature of Eq. 2.
* :func:`pair` -- Eq. 3 summed in the order of Alg. 5 (Neumaier sums).
* :func:`pair_anglesum` -- the angle-summation evaluation of the appendix (Alg. 7).
* :func:`direct_sum` -- :func:`pair` over a pair list, threaded over pairs.
* :func:`loop_flags` -- the zero-length-segment test of Alg. 3 plus finiteness.
* :func:`aabb_pairs` -- brute-force potential link search (Alg. 2 semantics).
* :func:`crossings` -- brute-force signed crossing count (Sec. 2.1).
* :func:`verify` -- the before/after comparison of two sparse linking
  matrices (Sec. 3.1, "Fast Verification").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lk_oracle.c")
_LIB = os.path.join(_HERE, "liblkoracle.so")
_lock = threading.Lock()
_lib = None

# Flag bits reported by loop_flags (same meaning as the library's flags).
FLAG_NONFINITE = 4
FLAG_BADLOOP = 16


# Optimisation without any change of FP semantics: no fast-math, no
# contraction into fused multiply-adds, so every operation rounds as written.
CFLAGS = ["-O3", "-fno-fast-math", "-ffp-contract=off"]


def build(force: bool = True) -> str:
    """Compile lk_oracle.c into liblkoracle.so with gcc and CFLAGS."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", *CFLAGS, "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        d, i64, i32, p = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.lko_term.restype = d
        lib.lko_term.argtypes = [p, p, p, p]
        lib.lko_term_mid.restype = d
        lib.lko_term_mid.argtypes = [p, p, p, p]
        lib.lko_pair.restype = d
        lib.lko_pair.argtypes = [p, i64, p, i64]
        lib.lko_pair_anglesum.restype = d
        lib.lko_pair_anglesum.argtypes = [p, i64, p, i64]
        lib.lko_direct_sum.restype = ctypes.c_int
        lib.lko_direct_sum.argtypes = [p, p, i32, p, i64, p, p, ctypes.c_int]
        lib.lko_loop_flags.restype = ctypes.c_int
        lib.lko_loop_flags.argtypes = [p, p, i32, d, p]
        lib.lko_aabb_pairs.restype = i64
        lib.lko_aabb_pairs.argtypes = [p, p, i32, p, i64]
        lib.lko_verify.restype = i64
        lib.lko_verify.argtypes = [p, p, i64, p, p, i64, p, i64]
        lib.lko_crossings.restype = d
        lib.lko_crossings.argtypes = [p, i64, p, i64, p, ctypes.POINTER(ctypes.c_int)]
        lib.lko_bh_pair.restype = d
        lib.lko_bh_pair.argtypes = [p, i64, p, i64, d, ctypes.c_int, i64, i64,
                                    ctypes.POINTER(ctypes.c_double)]
        lib.lko_bh_far_pieces.restype = d
        lib.lko_bh_far_pieces.argtypes = [p, i64, i64, i64, p, i64, i64, i64, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_double)]
        lib.lko_discretize.restype = i64
        lib.lko_discretize.argtypes = [p, p, i32, ctypes.c_int, p, i64, d, ctypes.c_int,
                                       ctypes.c_uint32, p, p, i64, p]
        lib.lko_bh_node_moments.restype = None
        lib.lko_bh_node_moments.argtypes = [p, i64, i64, i64, p]
        lib.lko_set_mutation.restype = None
        lib.lko_set_mutation.argtypes = [ctypes.c_int]
        _lib = lib
        return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_mutation(m: int) -> None:
    """Plant a deliberate mistake in the oracle (tests of the pins only).

    1 drop a term of D1, 2 wrong sign in the second arctangent, 3 wrong vertex
    index in c, 4 transposed difference vectors, 5 open (non-cyclic) loop,
    6 wrong normalisation (4 pi instead of 2 pi).  0 restores the oracle.
    """
    _load().lko_set_mutation(int(m))


def term(lj, lj1, ki, ki1) -> float:
    """Eq. 4 for segment (lj, lj1) of gamma_1 and segment (ki, ki1) of gamma_2."""
    v = [_f64(x).reshape(3) for x in (lj, lj1, ki, ki1)]
    return _load().lko_term(*[_ptr(x) for x in v])


def term_midpoint(lj, lj1, ki, ki1) -> float:
    """Midpoint quadrature of Eq. 2 for one segment pair."""
    v = [_f64(x).reshape(3) for x in (lj, lj1, ki, ki1)]
    return _load().lko_term_mid(*[_ptr(x) for x in v])


def pair(L, K) -> float:
    """Linking number of closed polylines L (gamma_1) and K (gamma_2), Alg. 5."""
    L = _f64(L).reshape(-1, 3)
    K = _f64(K).reshape(-1, 3)
    return _load().lko_pair(_ptr(L), L.shape[0], _ptr(K), K.shape[0])


def pair_anglesum(L, K) -> float:
    """Same value via the angle-summation form of Alg. 7."""
    L = _f64(L).reshape(-1, 3)
    K = _f64(K).reshape(-1, 3)
    return _load().lko_pair_anglesum(_ptr(L), L.shape[0], _ptr(K), K.shape[0])


def direct_sum(xyz, offsets, pairs, nthreads: int | None = None):
    """Real and integer linking numbers for every pair (loop pairs[p,0] is gamma_1).

    ``xyz`` may be float32 or float64; float32 values are promoted exactly.
    Returns ``(real float64[P], int int32[P])``; invalid pairs give NaN and
    INT32_MIN.
    """
    xyz = _f64(xyz).reshape(-1, 3)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32)).reshape(-1, 2)
    n = pr.shape[0]
    real = np.zeros(n, dtype=np.float64)
    lk = np.zeros(n, dtype=np.int32)
    if nthreads is None:
        try:
            nthreads = len(os.sched_getaffinity(0))
        except AttributeError:
            nthreads = os.cpu_count() or 1
        nthreads = min(nthreads, 16)
    rc = _load().lko_direct_sum(_ptr(xyz), _ptr(off), off.shape[0] - 1, _ptr(pr), n, _ptr(real),
                                _ptr(lk), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return real, lk


def loop_flags(xyz, offsets, eps: float):
    """Per-loop flags: FLAG_BADLOOP (<3 vertices or a segment shorter than
    eps * mean |coordinate|), FLAG_NONFINITE (NaN/Inf coordinate)."""
    xyz = _f64(xyz).reshape(-1, 3)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    out = np.zeros(off.shape[0] - 1, dtype=np.uint32)
    _load().lko_loop_flags(_ptr(xyz), _ptr(off), off.shape[0] - 1, float(eps), _ptr(out))
    return out


def aabb_pairs(xyz, offsets):
    """All i<j with overlapping closed AABBs, lexicographic, as int32[P,2]."""
    xyz = _f64(xyz).reshape(-1, 3)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    lib = _load()
    n = lib.lko_aabb_pairs(_ptr(xyz), _ptr(off), off.shape[0] - 1, None, 0)
    out = np.zeros((max(n, 1), 2), dtype=np.int32)
    lib.lko_aabb_pairs(_ptr(xyz), _ptr(off), off.shape[0] - 1, _ptr(out), n)
    return out[:n]


def verify(pairs, lk, exp_pairs, exp_lk):
    """Mismatches between the current (pairs, lk) and the expected
    (exp_pairs, exp_lk) sparse matrices, both sorted by (i, j); a pair missing
    on one side counts as 0 there.  Returns int32[m, 4] rows
    (i, j, current, expected) in pair order."""
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32)).reshape(-1, 2)
    v = np.ascontiguousarray(np.asarray(lk, dtype=np.int32)).reshape(-1)
    ep = np.ascontiguousarray(np.asarray(exp_pairs, dtype=np.int32)).reshape(-1, 2)
    ev = np.ascontiguousarray(np.asarray(exp_lk, dtype=np.int32)).reshape(-1)
    lib = _load()
    m = lib.lko_verify(_ptr(pr), _ptr(v), pr.shape[0], _ptr(ep), _ptr(ev), ep.shape[0], None, 0)
    out = np.zeros((max(m, 1), 4), dtype=np.int32)
    lib.lko_verify(_ptr(pr), _ptr(v), pr.shape[0], _ptr(ep), _ptr(ev), ep.shape[0], _ptr(out), m)
    return out[:m]


def crossings(L, K, R):
    """Half the signed crossing count of L and K viewed along z after x -> R x.

    Returns ``(value, degenerate)``; when ``degenerate`` the frame is not a
    regular projection for this pair and another frame must be drawn.
    """
    L = _f64(L).reshape(-1, 3)
    K = _f64(K).reshape(-1, 3)
    R = _f64(R).reshape(3, 3)
    deg = ctypes.c_int(0)
    v = _load().lko_crossings(_ptr(L), L.shape[0], _ptr(K), K.shape[0], _ptr(R), ctypes.byref(deg))
    return v, bool(deg.value)


def crossings_random(L, K, seed: int = 0, tries: int = 20) -> float:
    """Crossing count in a seeded random frame (QR of a Gaussian matrix),
    drawing again whenever the projection is not regular."""
    rng = np.random.default_rng(seed)
    for _ in range(tries):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        v, deg = crossings(L, K, q)
        if not deg:
            return v
    raise RuntimeError("no regular projection found")


def bh_pair(L, K, beta: float, order: int = 2, leaf: int = 64, arity: int = 8):
    """Barnes-Hut linking number of loops L (curve 1) and K (curve 2), Alg. 6:
    trees of ``leaf`` consecutive segments per leaf and ``arity`` children per
    node, far field to ``order`` (1 dipole, 2 quadrupole).  Returns
    ``(value, error_estimate)``."""
    L = _f64(L).reshape(-1, 3)
    K = _f64(K).reshape(-1, 3)
    err = ctypes.c_double(0.0)
    v = _load().lko_bh_pair(_ptr(L), L.shape[0], _ptr(K), K.shape[0], float(beta), int(order),
                            int(leaf), int(arity), ctypes.byref(err))
    return v, err.value


def bh_pair_adaptive(L, K, beta_init: float = 2.0, beta_max: float = 10.0, target: float = 0.2,
                     order: int = 2, leaf: int = 64, arity: int = 8):
    """The adaptive beta of Sec. 3.4.4: Barnes-Hut at beta_init; from its
    next-order error estimate E, beta_t = (E / target)^(1/4) beta_init; if
    beta_t > beta_init, evaluate again at min(beta_t, beta_max).  Returns
    ``(value, first_estimate, beta_used)``."""
    v, e = bh_pair(L, K, beta_init, order, leaf, arity)
    bt = (e / target) ** 0.25 * beta_init
    if bt > beta_init:
        beta = min(bt, beta_max)
        v, _ = bh_pair(L, K, beta, order, leaf, arity)
        return v, e, beta
    return v, e, beta_init


def bh_node_moments(P, a: int, b: int):
    """Centre, R and moments (c_M, C_D, C_Q) of the node covering segments
    [a, b) of loop P, computed directly from its segments."""
    P = _f64(P).reshape(-1, 3)
    out = np.zeros(43)
    _load().lko_bh_node_moments(_ptr(P), P.shape[0], int(a), int(b), _ptr(out))
    return {"c": out[0:3], "R": out[3], "M": out[4:7], "D": out[7:16].reshape(3, 3),
            "Q": out[16:43].reshape(3, 3, 3)}


def bh_far_pieces(P1, a1: int, b1: int, P2, a2: int, b2: int, order: int = 2):
    """Far-field estimate of the Gauss integral between segments [a1, b1) of
    loop P1 and [a2, b2) of loop P2, and the exact Eq. 4 sum over the same
    segment pairs: ``(estimate, exact)``."""
    P1 = _f64(P1).reshape(-1, 3)
    P2 = _f64(P2).reshape(-1, 3)
    ex = ctypes.c_double(0.0)
    v = _load().lko_bh_far_pieces(_ptr(P1), P1.shape[0], int(a1), int(b1), _ptr(P2), P2.shape[0],
                                  int(a2), int(b2), int(order), ctypes.byref(ex))
    return v, ex.value


FLAG_INTERSECT = 64
DZ_BSPLINE = 0
DZ_POLYLINE = 1


def discretize(ctrl, cp_offsets, pairs, kind: int = DZ_BSPLINE,
               eps: float = float(np.finfo(np.float64).eps), max_passes: int = 64):
    """Alg. 3 (Sec. 3.3): closed curves (``kind`` DZ_BSPLINE: uniform cubic
    B-spline control points; DZ_POLYLINE: vertices) given as ``ctrl`` [N][3]
    and ``cp_offsets`` [L+1], refined against the candidate ``pairs`` until no
    two pieces of a pair's loops have overlapping boxes.  Returns
    ``(xyz [V][3] float64, offsets [L+1] int64, loop_flags [L] uint32)``; flag
    16 = invalid loop (fewer than 3 points, non-finite, or a piece shorter
    than eps * xi), FLAG_INTERSECT = refinement reached eps * xi (curves
    within about that distance) or did not finish in ``max_passes``."""
    ctrl = _f64(ctrl).reshape(-1, 3)
    off = np.ascontiguousarray(cp_offsets, dtype=np.int64)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    L = off.shape[0] - 1
    out_off = np.zeros(L + 1, dtype=np.int64)
    flags = np.zeros(max(L, 1), dtype=np.uint32)
    lib = _load()
    args = (_ptr(ctrl), _ptr(off), L, int(kind), _ptr(pr), pr.shape[0], float(eps),
            int(max_passes), FLAG_INTERSECT)
    n = lib.lko_discretize(*args, None, _ptr(out_off), 0, _ptr(flags))
    if n < 0:
        raise MemoryError("oracle discretization failed")
    xyz = np.zeros((max(n, 1), 3))
    lib.lko_discretize(*args, _ptr(xyz), _ptr(out_off), n, _ptr(flags))
    return xyz[:n], out_off, flags[:L]

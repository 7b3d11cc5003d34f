"""The sign rule of the merged per-term arctangent (Eq. 4), on the CPU.

The direct-sum kernel evaluates both arctangents of Eq. 4 as one angle,
theta = arg((d1 + i p)(d2 + i p)), with the walk algebra of its hot loop
(norms and dot products carried from the previous step of loop A).  This file
repeats that algebra for one segment pair in numpy FP32 (no fused
multiply-adds) and checks it against the oracle's Eq. 4 on perpendicular
segments that pass within h of each other with the crossing near the diagonal
a-c of the pair's quadrilateral, where d1 and d2 both vanish.  Taking the
angle's sign from p(d1 + d2) there turns about a quarter of the terms into
errors of exactly one unit; taking it from p, as the kernel does, leaves an
error that grows like eps |s| / h and stays far from one.
"""
import numpy as np

import oracle

f32 = np.float32


def _dot(a, b):
    return f32(f32(f32(a[0] * b[0]) + f32(a[1] * b[1])) + f32(a[2] * b[2]))


def _cross(a, b):
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]], f32)


def walk_term(lj, lj1, k0, k1, sign_from_p: bool) -> float:
    """Eq. 4 for segment (lj, lj1) against (k0, k1) through the kernel's walk:
    the start of the walk at lj (walk_init), then one step to lj1 (walk_step)."""
    lj, lj1, k0, k1 = (np.asarray(v, f32) for v in (lj, lj1, k0, k1))
    s0 = k1 - k0
    V0, V1 = lj - k0, lj - k1
    N0, N1 = np.sqrt(_dot(V0, V0)), np.sqrt(_dot(V1, V1))
    E0 = N0 * N1 + _dot(V0, V1)
    G0 = _dot(s0, V0)
    v0, v1 = lj1 - k0, lj1 - k1
    n20 = _dot(v0, v0)
    n0, n1 = np.sqrt(n20), np.sqrt(_dot(v1, v1))
    vert0, vert1 = _dot(V0, v0), _dot(V1, v1)
    p = _dot(s0, _cross(V0, lj1 - lj))
    ca = vert0 - G0
    f = n0 * n1 + (n20 - _dot(s0, v0))
    d1 = n1 * E0 + vert1 * N0 + ca * N1
    d2 = N0 * f + vert0 * n1 + ca * n0
    y = p * abs(d1 + d2) if sign_from_p else p * (d1 + d2)
    x = d1 * d2 - p * p
    return float(np.arctan2(f32(y), f32(x))) / (2 * np.pi)


def _cases(rng, h_rel, n):
    for _ in range(n):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        c = rng.uniform(-3, 3, 3)
        ln = rng.uniform(0.05, 0.2)
        ta = rng.uniform(0.2, 0.8)
        tb = ta + rng.choice([0.0, 1e-5, 1e-3])
        pts = [np.array([-ta * ln, 0, 0]), np.array([(1 - ta) * ln, 0, 0]),
               np.array([0, -tb * ln, h_rel * ln]), np.array([0, (1 - tb) * ln, h_rel * ln])]
        yield [np.asarray(c + q @ v, f32).astype(np.float64) for v in pts]


def test_walk_algebra_matches_eq4_away_from_contact():
    rng = np.random.default_rng(1)
    for _ in range(300):
        pts = rng.uniform(-1, 1, (4, 3))
        ref = oracle.term(*pts)
        assert abs(walk_term(*pts, True) - ref) < 2e-5
        # away from contact both sign rules agree
        assert walk_term(*pts, True) == walk_term(*pts, False)


def test_sign_from_p_near_contact():
    rng = np.random.default_rng(0)
    for h_rel, worst_new in ((1e-2, 1e-4), (1e-3, 1e-3), (1e-4, 1e-2), (1e-5, 0.1)):
        bad_old = bad_new = 0
        err_new = 0.0
        for pts in _cases(rng, h_rel, 400):
            ref = oracle.term(*pts)
            bad_old += abs(walk_term(*pts, False) - ref) > 0.5
            e = abs(walk_term(*pts, True) - ref)
            bad_new += e > 0.5
            err_new = max(err_new, e)
        assert bad_new == 0, h_rel
        assert err_new < worst_new, (h_rel, err_new)
        if h_rel <= 1e-4:
            # the old rule fails here: whole-unit errors the refit rule cannot see
            assert bad_old > 20, (h_rel, bad_old)

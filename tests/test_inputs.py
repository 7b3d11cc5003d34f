"""Construction rules of the seeded generators, checked against the oracle.

The generators state the linking numbers their shapes are built to have; these
tests compare those statements with the oracle on instances small enough for
it, and check the size/shape recipes of the workloads.
"""
import numpy as np

import oracle
from paper_2106_12655_amd import inputs as I


def _check_against_oracle(ls, pairs=None):
    if pairs is None:
        pairs = oracle.aabb_pairs(ls.xyz, ls.offsets)
    real, lk = oracle.direct_sum(ls.xyz, ls.offsets, pairs)
    exp = ls.expected_for(pairs)
    assert np.array_equal(lk, exp), np.nonzero(lk != exp)
    assert np.max(np.abs(real - np.round(real))) < 1e-8
    return pairs, real


def test_ring_grid_recipe_and_links():
    ls = I.ring_grid(0)
    assert ls.n_loops == 64 and np.all(ls.sizes == 32) and ls.xyz.dtype == np.float64
    pairs, _ = _check_against_oracle(ls)
    assert len(pairs) == 105
    assert len(ls.exp_pairs) == 56
    assert set(np.unique(ls.exp_lk).tolist()) == {-1, 1}


def test_ring_grid_seeds_differ_but_links_do_not():
    a, b = I.ring_grid(1), I.ring_grid(2)
    assert not np.array_equal(a.xyz, b.xyz)
    _check_against_oracle(a)
    _check_against_oracle(b)


def test_chainmail_patch_links():
    ls = I.chainmail(0, rows=6, cols=7)
    assert ls.xyz.dtype == np.float32
    pairs, _ = _check_against_oracle(ls)
    # interior rings link exactly four neighbours
    deg = np.zeros(ls.n_loops, int)
    for i, j in ls.exp_pairs:
        deg[i] += 1
        deg[j] += 1
    interior = [r * 7 + c for r in range(1, 5) for c in range(1, 6)]
    assert np.all(deg[interior] == 4)
    # the 45 degree sheet rotation adds unlinked candidates
    assert len(pairs) > 2 * len(ls.exp_pairs)


def test_chainmail_pull_through_unlinks_only_selected():
    # edge rings slid out of the sheet: exactly their two links become 0, with
    # the serving noise level (0.05) on the wider row pitch
    rows, cols = 6, 7
    pick = [2, 5, (rows - 1) * cols + 1, (rows - 1) * cols + 4, 3 * cols + 2]  # last one is interior
    ls = I.chainmail(3, rows=rows, cols=cols, row_pitch=1.25, sigma=0.05, noise_seed=8,
                     pulled_rings=pick)
    assert len(ls.meta["pulled"]) == 8
    base = I.chainmail(3, rows=rows, cols=cols, row_pitch=1.25, sigma=0.0)
    _check_against_oracle(ls)  # every candidate pair as constructed
    gone = {tuple(x) for x in base.exp_pairs.tolist()} - {tuple(x) for x in ls.exp_pairs.tolist()}
    assert gone == {tuple(x) for x in ls.meta["pulled"].tolist()}
    for i, j in gone:  # pulled pairs are unlinked (their boxes may no longer overlap)
        assert abs(oracle.pair(ls.loop(i), ls.loop(j))) < 1e-9


def test_chainmail_serving_noise_is_safe_on_wide_pitch():
    # per-vertex noise 0.05 keeps every construction value on the 1.25 pitch
    ls = I.chainmail(4, rows=12, cols=12, nseg=48, row_pitch=1.25, sigma=0.05, noise_seed=2)
    _check_against_oracle(ls)


def test_chainmail_full_size_recipe():
    ls = I.chainmail(0)
    assert ls.n_loops == 14000 and np.all(ls.sizes == 64)
    pairs = oracle.aabb_pairs(ls.xyz, ls.offsets)
    assert 60000 < len(pairs) < 80000
    assert 27000 < len(ls.exp_pairs) < 29000
    assert abs(I.terms(ls.sizes, pairs) - 2.8e8) < 0.1e8


def test_knit_small_tubes():
    ls = I.knit(0, n_loops=30, cp_max=48, per_span=4, linked_fraction=0.5)
    _check_against_oracle(ls)
    assert np.any(ls.exp_lk != 0)


def test_knit_tube_patterns():
    rows, exp = I.knit_tube(6, 3, per_span=6, pattern="uniform")
    xyz = np.vstack(rows)
    off = np.concatenate([[0], np.cumsum([len(r) for r in rows])])
    real, lk = oracle.direct_sum(xyz, off, [[0, 1], [1, 2], [0, 2]])
    assert lk.tolist() == [6, 6, 0] and exp == {(0, 1): 6, (1, 2): 6}
    rows, exp = I.knit_tube(6, 3, per_span=6, flip={(1, 0)})
    xyz = np.vstack(rows)
    real, lk = oracle.direct_sum(xyz, off, [[0, 1], [1, 2]])
    assert lk.tolist() == [exp[(0, 1)], exp[(1, 2)]] and exp[(0, 1)] == -2


def test_knit_full_size_recipe():
    ls = I.knit(0)
    assert ls.n_loops == 2000
    s = ls.sizes
    assert s.min() >= 512 and s.max() <= 16384 and s.max() / s.min() >= 16
    pairs = oracle.aabb_pairs(ls.xyz, ls.offsets)
    assert len(pairs) > 5000


def test_winding_pairs_small():
    for lk in (-3, 0, 2, 5):
        C, D, v = I.winding_pair(11 + lk, 2500, 2600, lk, step=0.02, rho=0.15)
        assert v == lk
        assert abs(oracle.pair(C, D) - lk) < 1e-8


def test_long_pairs_recipe_small():
    ls = I.long_pairs(0, n_pairs=3, n_min=1500, n_max=2500, step=0.02, rho=0.15, dtype=np.float64)
    _check_against_oracle(ls, ls.pairs)
    assert len(ls.pairs) == 3


def test_generators_are_deterministic():
    a, b = I.chainmail(5, rows=3, cols=3), I.chainmail(5, rows=3, cols=3)
    assert np.array_equal(a.xyz, b.xyz)
    a, b = I.knit(5, n_loops=10, cp_max=32, per_span=2), I.knit(5, n_loops=10, cp_max=32, per_span=2)
    assert np.array_equal(a.xyz, b.xyz)


def test_winding_pair_full_length_coarse():
    # the long-loop recipe at its real length (1000 units) but coarse steps:
    # the petal outline keeps the construction rule Lk = number of turns
    C, D, v = I.winding_pair(104, 20000, 21000, -4, step=0.05, rho=0.1)
    xyz = np.vstack([C, D])
    real, lk = oracle.direct_sum(xyz, [0, len(C), len(C) + len(D)], [[0, 1]])
    assert lk[0] == v == -4 and abs(real[0] - v) < 1e-8


def test_near_contact_construction():
    # perpendicular segments h apart: -1 when B passes outside A's segment, 0
    # when it passes inside (both of its crossings of A's plane are in A)
    h = [1e-1, 1e-2, -1e-2, 1e-4, -1e-4]
    ls = I.near_contact(h, 0.4, 0.6, seed=3)
    _check_against_oracle(ls, ls.pairs)
    assert ls.expected_for(ls.pairs).tolist() == [-1, -1, 0, -1, 0]
    # the closest points of the two last segments are h apart
    for k, hk in enumerate(ls.meta["h"]):
        A, B = ls.loop(2 * k), ls.loop(2 * k + 1)
        sa, sb = A[0] - A[-1], B[0] - B[-1]
        n = np.cross(sa, sb)
        assert abs(abs((B[-1] - A[-1]) @ n) / np.linalg.norm(n) - abs(hk)) < 1e-12


def test_near_parallel_construction():
    ls = I.near_parallel([1e-1, 1e-2, 1e-4, 1e-4], [0.0, 1e-3, 0.0, 1e-4], seed=4)
    _check_against_oracle(ls, ls.pairs)
    assert np.all(ls.expected_for(ls.pairs) == -1)

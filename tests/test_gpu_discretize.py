"""Discretization on the GPU (lk_discretize, Sec. 3.3, Alg. 3) against the oracle.

Both sides build the same Bezier pieces, test the same closed-interval box
overlaps, split with the same de Casteljau halving in FP64 (no fused
multiply-adds) and keep parameter order, so vertices, offsets and loop flags
must be bitwise equal.  xi is summed in a different order on the two sides;
it only decides the degenerate-length flags, which none of the regular cases
come near.  At the full knit size the oracle is too slow, so the output is
checked by properties that hold at any size: every vertex is a curve point at
a dyadic parameter in order, and the linking numbers of the polylines are the
construction's.
"""
import numpy as np
import pytest

import oracle
from paper_2106_12655_amd import inputs as I
from test_oracle_pins import (_bspline_at, _dyadic_parse, _pack_loops, _polyline_at,
                              _square_triangle, _through_arc)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dctx():
    import paper_2106_12655_amd as lk
    c = lk.Context(0)
    yield c
    c.close()


def _gpu(c, ctrl, off, pairs, kind="bspline", capacity=None):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(ctrl, dtype=np.float64)).cuda()
    o = torch.from_numpy(np.ascontiguousarray(off, dtype=np.int64)).cuda()
    p = torch.from_numpy(np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))).cuda()
    xyz, off_out, flags, info = c.discretize(x, o, p, kind, capacity)
    torch.cuda.synchronize()
    return (xyz.cpu().numpy(), off_out.cpu().numpy(), flags.cpu().numpy().view(np.uint32), info)


def _compare(c, ctrl, off, pairs, kind="bspline", label="", max_passes=64):
    ok = oracle.DZ_POLYLINE if kind == "polyline" else oracle.DZ_BSPLINE
    ox, oo, of = oracle.discretize(ctrl, off, pairs, kind=ok, max_passes=max_passes)
    gx, go, gf, info = _gpu(c, ctrl, off, pairs, kind)
    print("%s: N_I %d -> N_D %d in %d passes, flags %s" % (
        label, len(ctrl), go[-1], info["passes"], np.unique(gf)), flush=True)
    assert np.array_equal(go, oo), label
    assert np.array_equal(gf, of), label
    assert gx.shape == ox.shape, label
    assert np.array_equal(gx.view(np.uint64), ox.view(np.uint64)), label
    assert info["vertices"] == go[-1] and info["input_spans"] == len(ctrl)
    return gx, go, gf, info


def _knit_ctrl(seed, n_loops, cp_max=128):
    k = I.knit(seed, n_loops=n_loops, cp_max=cp_max, per_span=0, dtype=np.float64)
    return k, oracle.aabb_pairs(k.xyz, k.offsets)


def test_bitwise_parity_knit(dctx):
    for seed, nl, cpm in ((0, 12, 64), (1, 40, 128), (2, 90, 512)):
        k, pr = _knit_ctrl(seed, nl, cpm)
        _compare(dctx, k.xyz, k.offsets, pr, label="knit %d rows (seed %d)" % (nl, seed))


def test_bitwise_parity_small_constructions(dctx):
    loops = _through_arc()
    xyz, off = _pack_loops(loops)
    for pairs in ([[0, 1]], [[1, 0]], []):
        _compare(dctx, xyz, off, pairs, label="through-arc %s" % pairs)
    loops, _ = I.knit_tube(4, 3, per_span=0, pattern="uniform")
    xyz, off = _pack_loops(loops)
    _compare(dctx, xyz, off, [[0, 1], [1, 2], [0, 2]], label="knit tube")
    sq, tri = _square_triangle()
    xyz, off = _pack_loops([sq, tri])
    _compare(dctx, xyz, off, [[0, 1]], kind="polyline", label="square-triangle")


def test_bitwise_parity_polyline_grid(dctx):
    g = I.ring_grid(3, rows=4, cols=4, nseg=12)
    xyz = np.asarray(g.xyz, np.float64)
    pr = oracle.aabb_pairs(xyz, g.offsets)
    _compare(dctx, xyz, g.offsets, pr, kind="polyline", label="ring grid 4x4, 12 segments")
    # the same rings as closed B-splines (control polygons)
    _compare(dctx, xyz, g.offsets, pr, label="ring grid as B-splines")


def test_edge_cases(dctx):
    """Invalid pairs, invalid loops (fewer than 3 points, NaN, zero-length
    span, empty), touching curves and the pass limit match the oracle."""
    sq, tri = _square_triangle()
    tri_touch = np.array([[1.0, 0, 0], [3, 0.5, 1], [3, -0.5, -1]])
    rep = sq.copy()
    rep[2] = rep[1]
    nan = sq.copy()
    nan[1, 2] = np.nan
    loops = [sq, tri_touch, rep + [0, 0, 0.5], sq[:2] + [0, 0, 2], tri + [0, 0, 0.1]]
    xyz, off = _pack_loops(loops)
    # an empty loop at the end
    off = np.concatenate([off, off[-1:]])
    pairs = [[0, 1], [0, 2], [0, 3], [0, 4], [0, 0], [0, 9], [-1, 2], [5, 4]]
    gx, go, gf, info = _compare(dctx, xyz, off, pairs, kind="polyline", label="edge cases")
    assert gf[0] & oracle.FLAG_INTERSECT and gf[1] & oracle.FLAG_INTERSECT
    assert gf[2] == 16 and gf[3] == 16 and gf[5] == 16 and gf[4] == 0
    # a NaN coordinate: its loop is invalid (and xi is NaN for the call)
    xyz, off = _pack_loops([sq, nan, tri])
    gx, go, gf, info = _compare(dctx, xyz, off, [[0, 1], [0, 2], [1, 2]], kind="polyline",
                                label="NaN loop")
    assert gf[1] == 16 and gf[0] == 0 and gf[2] == 0
    # the pass limit
    import paper_2106_12655_amd as lk
    loops, _ = I.knit_tube(4, 3, per_span=0, pattern="uniform")
    xyz, off = _pack_loops(loops)
    try:
        dctx.set_option(lk._lib.OPT_DZ_MAX_PASSES, 1)
        gx, go, gf, info = _compare(dctx, xyz, off, [[0, 1]], label="one pass", max_passes=1)
        assert info["passes"] == 1 and info["unfinished"] > 0
        assert gf[0] & oracle.FLAG_INTERSECT and gf[1] & oracle.FLAG_INTERSECT and gf[2] == 0
    finally:
        dctx.set_option(lk._lib.OPT_DZ_MAX_PASSES, 64)
    # no pairs at all, and a single loop
    _compare(dctx, xyz, off, [], label="no pairs")
    _compare(dctx, loops[0], [0, len(loops[0])], [], label="one loop")


def test_long_loops_many_groups(dctx):
    """Two loops of 5,000 control points each (79 groups of 64 pieces, so a
    work item walks the other loop's groups in two chunks of 64), wound
    around each other three times at a distance close to the control
    spacing: refined in several passes, bitwise equal to the oracle for
    both curve kinds, and still linked three times."""
    r = I.winding_pair(5, 15000, 15000, 3, step=0.03, rho=0.04)
    a, b = r[0][::3], r[1][::3]
    ctrl = np.vstack([a, b])
    off = np.array([0, len(a), len(a) + len(b)], np.int64)
    for kind in ("bspline", "polyline"):
        gx, go, gf, info = _compare(dctx, ctrl, off, [[0, 1]], kind=kind,
                                    label="winding pair 5000 + 5000, %s" % kind)
        assert go[-1] > len(ctrl) and info["passes"] >= 2
        assert abs(oracle.pair(gx[go[0]:go[1]], gx[go[1]:go[2]]) - 3.0) < 1e-6


def test_pair_order_capacity_and_repeat(dctx):
    import paper_2106_12655_amd as lk
    k, pr = _knit_ctrl(4, 30)
    a = _gpu(dctx, k.xyz, k.offsets, pr)
    rng = np.random.default_rng(0)
    perm = pr[rng.permutation(len(pr))][:, ::-1]
    b = _gpu(dctx, k.xyz, k.offsets, np.vstack([perm, pr[:5]]))
    c = _gpu(dctx, k.xyz, k.offsets, pr)
    for x, y in ((a, b), (a, c)):
        assert np.array_equal(x[0].view(np.uint64), y[0].view(np.uint64))
        assert np.array_equal(x[1], y[1]) and np.array_equal(x[2], y[2])
    # too small a buffer: offsets and flags written, LK_ECAPACITY with the size
    with pytest.raises(lk.LkError) as e:
        _gpu(dctx, k.xyz, k.offsets, pr, capacity=10)
    assert e.value.status == lk._lib.ECAPACITY
    # offsets that decrease are rejected before any kernel uses them
    bad = k.offsets.copy()
    bad[3] = bad[5]
    with pytest.raises(lk.LkError) as e:
        _gpu(dctx, k.xyz, bad, pr)
    assert e.value.status == lk._lib.EINVAL


def test_full_knit_properties(dctx):
    """The 2000-row knit (314k control points): vertices of sampled rows are
    curve points at dyadic parameters in order, no loop is flagged, and the
    FP64 direct sum of the polylines gives the construction's linking number
    for every candidate pair (where the polyline through the knots is wrong
    for the linked rows)."""
    import torch
    k = I.knit(0, per_span=0, dtype=np.float64)
    x = torch.from_numpy(k.xyz).cuda()
    o = torch.from_numpy(k.offsets).cuda()
    pr = dctx.build_pairs(x, o)
    xyz, off, flags, info = dctx.discretize(x, o, pr)
    pairs = pr.cpu().numpy()
    print("knit 2000 rows: %d pairs, N_I %d -> N_D %d, %d passes" % (
        len(pairs), len(k.xyz), info["vertices"], info["passes"]), flush=True)
    assert (flags.cpu().numpy() == 0).all() and info["unfinished"] == 0
    real, lk_int, pf = dctx.direct_sum(xyz, off, pr, "plain")
    exp = k.expected_for(pairs)
    assert np.array_equal(lk_int.cpu().numpy(), exp)
    assert (exp != 0).sum() > 0
    hx, ho = xyz.cpu().numpy(), off.cpu().numpy()
    rng = np.random.default_rng(1)
    for i in rng.choice(k.n_loops, 12, replace=False):
        r = _dyadic_parse(k.loop(i), hx[ho[i]:ho[i + 1]], _bspline_at)
        assert not isinstance(r, str), "row %d: %s" % (i, r)
    # the oracle on sampled pairs of the GPU polylines
    for p in rng.choice(len(pairs), 8, replace=False):
        i, j = pairs[p]
        v = oracle.pair(hx[ho[i]:ho[i + 1]], hx[ho[j]:ho[j + 1]])
        assert abs(v - exp[p]) < 1e-6

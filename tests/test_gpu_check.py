"""The direct sum fused with the certificate check (lk_direct_sum_check).

Sec. 3.1 ("Fast Verification") compares a state's linking numbers with stored
ones and may stop at the first failure.  Checks: the fused call returns the
same values as lk_direct_sum and counts exactly the planted mismatches; with
early exit it stops (SKIPPED pairs carry no value) and every pair it did
finish is still exact; counts reset between calls and graph replays.
"""
import numpy as np
import pytest

import oracle
from paper_2106_12655_amd import inputs as I

pytestmark = pytest.mark.gpu


def _setup(ls):
    import torch
    xyz = torch.from_numpy(np.ascontiguousarray(ls.xyz)).cuda()
    off = torch.from_numpy(np.ascontiguousarray(ls.offsets)).cuda()
    return xyz, off


@pytest.mark.parametrize("mode", ["mixed", "plain"])
def test_check_counts_planted_mismatches(ctx, mode):
    import torch
    import paper_2106_12655_amd as lk
    ls = I.chainmail(3, rows=20, cols=20)
    pairs = oracle.aabb_pairs(ls.xyz, ls.offsets)
    exp = ls.expected_for(pairs)
    xyz, off = _setup(ls)
    pr = torch.from_numpy(pairs).cuda()
    real0, lk0, fl0 = [t.cpu().numpy() for t in ctx.direct_sum(xyz, off, pr, mode)]
    assert np.array_equal(lk0, exp)
    # all correct: no mismatch, identical outputs
    real, lkv, fl, nm = ctx.direct_sum_check(xyz, off, pr, torch.from_numpy(exp).cuda(), False, mode)
    torch.cuda.synchronize()
    assert int(nm.item()) == 0
    assert np.array_equal(real.cpu().numpy(), real0) and np.array_equal(lkv.cpu().numpy(), lk0)
    assert np.array_equal(fl.cpu().numpy(), fl0)
    # planted mismatches, no early exit: counted exactly, nothing skipped
    rng = np.random.default_rng(4)
    pick = rng.choice(len(exp), 17, replace=False)
    bad = exp.copy()
    bad[pick] += 1
    real, lkv, fl, nm = ctx.direct_sum_check(xyz, off, pr, torch.from_numpy(bad).cuda(), False, mode)
    torch.cuda.synchronize()
    assert int(nm.item()) == 17
    assert np.array_equal(lkv.cpu().numpy(), lk0)
    assert not np.any(fl.cpu().numpy() & lk.FLAG_SKIPPED)


@pytest.mark.parametrize("mode", ["mixed", "plain"])
def test_check_early_exit_stops_and_stays_exact(ctx, mode):
    import torch
    import paper_2106_12655_amd as lk
    ls = I.chainmail(0)  # 69k pairs: far more work than one round of the grid
    pairs = oracle.aabb_pairs(ls.xyz, ls.offsets)
    exp = ls.expected_for(pairs)
    xyz, off = _setup(ls)
    pr = torch.from_numpy(pairs).cuda()
    wrong = torch.from_numpy(exp + 1).cuda()  # every pair disagrees
    for rep in range(3):  # first call captures a graph, later ones replay it
        real, lkv, fl, nm = ctx.direct_sum_check(xyz, off, pr, wrong, True, mode)
        torch.cuda.synchronize()
        fl = fl.cpu().numpy().view(np.uint32)
        lkv = lkv.cpu().numpy()
        skipped = (fl & lk.FLAG_SKIPPED) != 0
        n = int(nm.item())
        print("%s rep %d: mismatches %d, skipped %d of %d" % (mode, rep, n, skipped.sum(), len(exp)),
              flush=True)
        assert n >= 1
        assert n == int((~skipped).sum())  # every finished pair disagrees by construction
        assert skipped.sum() > len(exp) // 4
        assert np.all(lkv[skipped] == lk.INT_INVALID)
        assert np.all(np.isnan(real.cpu().numpy()[skipped]))
        assert np.array_equal(lkv[~skipped], exp[~skipped])


def test_check_small_and_empty(ctx):
    import torch
    ls = I.ring_grid(0)
    pairs = oracle.aabb_pairs(ls.xyz, ls.offsets)
    exp = ls.expected_for(pairs)
    xyz, off = _setup(ls)
    pr = torch.from_numpy(pairs).cuda()
    _, lkv, _, nm = ctx.direct_sum_check(xyz, off, pr, torch.from_numpy(exp).cuda(), True, "mixed")
    torch.cuda.synchronize()
    assert int(nm.item()) == 0 and np.array_equal(lkv.cpu().numpy(), exp)
    # an invalid pair cannot be certified: it counts
    bad = pairs.copy()
    bad[0] = [3, 3]
    _, lkv, _, nm = ctx.direct_sum_check(xyz, off, torch.from_numpy(bad).cuda(),
                                         torch.from_numpy(exp).cuda(), False, "mixed")
    torch.cuda.synchronize()
    assert int(nm.item()) == 1
    # no pairs: the count is written as 0
    nm = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    out = (torch.empty(0, dtype=torch.float64, device="cuda"), torch.empty(0, dtype=torch.int32, device="cuda"),
           torch.empty(0, dtype=torch.int32, device="cuda"), nm)
    ctx.direct_sum_check(xyz, off, torch.zeros((0, 2), dtype=torch.int32, device="cuda"), e, True,
                         "mixed", out=out)
    torch.cuda.synchronize()
    assert int(nm.item()) == 0

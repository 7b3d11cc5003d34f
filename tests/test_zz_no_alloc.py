"""lk_direct_sum_noalloc (the entry point for callers that cannot allocate)
against lk_direct_sum on the same context: bitwise equal values, integers and
flags, on two calls in a row of which the second is smaller, in both modes
it supports; its limits are refused on the host."""
import numpy as np
import pytest

import oracle
from paper_2106_12655_amd import _lib
from paper_2106_12655_amd import inputs as I

pytestmark = pytest.mark.gpu


def _with_pairs(ls):
    ls.pairs = oracle.aabb_pairs(ls.xyz, ls.offsets).astype(np.int32)
    return ls


def _dev(ls):
    import torch
    xyz = torch.from_numpy(np.ascontiguousarray(ls.xyz)).cuda()
    off = torch.from_numpy(np.ascontiguousarray(ls.offsets)).cuda()
    pr = torch.from_numpy(np.ascontiguousarray(ls.pairs.reshape(-1, 2))).cuda()
    return xyz, off, pr


def _host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("mode", ["mixed", "plain"])
def test_noalloc_equals_direct_sum(mode):
    import torch
    import paper_2106_12655_amd as lk
    ctx = lk.Context(0)  # default options on both sides
    big = _with_pairs(I.chainmail(0))           # 14,000 loops x 64, FP32, ~69k pairs
    small = _with_pairs(I.ring_grid(1))         # 64 loops x 32, FP64, 105 pairs
    assert len(big.pairs) > 60000 and len(small.pairs) < len(big.pairs)
    for k, ls in enumerate((big, small)):
        xyz, off, pr = _dev(ls)
        print("noalloc %s: call %d, %d loops, %d pairs" % (mode, k, len(ls.offsets) - 1,
                                                          len(ls.pairs)), flush=True)
        a = ctx.direct_sum_noalloc(xyz, off, pr, mode)
        torch.cuda.synchronize()
        b = ctx.direct_sum(xyz, off, pr, mode)
        torch.cuda.synchronize()
        ra, la, fa = (_host(t) for t in a)
        rb, lb, fb = (_host(t) for t in b)
        assert np.array_equal(ra.view(np.uint64), rb.view(np.uint64)), "values differ"
        assert np.array_equal(la, lb), "integers differ"
        assert np.array_equal(fa, fb), "flags differ"
        assert np.array_equal(la, ls.expected_for(ls.pairs)), "integers differ from construction"
    # the smaller call's integers against the oracle as well
    oreal, olk = oracle.direct_sum(small.xyz, small.offsets, small.pairs)
    assert np.array_equal(la, olk)
    assert np.max(np.abs(ra - oreal)) <= (1e-6 if mode == "plain" else 1e-5)
    ctx.close()


def test_noalloc_null_flags_and_limits():
    import ctypes
    import torch
    import paper_2106_12655_amd as lk
    ctx = lk.Context(0)
    ls = _with_pairs(I.ring_grid(2))
    xyz, off, pr = _dev(ls)
    P = len(ls.pairs)
    ref = ctx.direct_sum(xyz, off, pr, "mixed")
    real = torch.full((P,), 7.0, dtype=torch.float64, device="cuda")
    lki = torch.full((P,), 7, dtype=torch.int32, device="cuda")
    ctx.direct_sum_noalloc(xyz, off, pr, "mixed", out=(real, lki, None))
    torch.cuda.synchronize()
    assert np.array_equal(_host(real), _host(ref[0]))
    assert np.array_equal(_host(lki), _host(ref[1]))
    # refused on the host, before anything is enqueued: outputs untouched
    real.fill_(7.0)
    torch.cuda.synchronize()
    st = ctx.lib.lk_direct_sum_noalloc(
        ctx.h, xyz.data_ptr(), _lib.F64, off.data_ptr(), len(ls.offsets) - 1, pr.data_ptr(),
        131073, _lib.MIXED, real.data_ptr(), lki.data_ptr(), None,
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.ECAPACITY
    assert b"131072" in ctx.lib.lk_last_error(ctx.h)
    st = ctx.lib.lk_direct_sum_noalloc(
        ctx.h, xyz.data_ptr(), _lib.F64, off.data_ptr(), 65537, pr.data_ptr(), P, _lib.MIXED,
        real.data_ptr(), lki.data_ptr(), None,
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.ECAPACITY
    with pytest.raises(lk.LkError):
        ctx.direct_sum_noalloc(xyz, off, pr, "crossings")
    torch.cuda.synchronize()
    assert np.all(_host(real) == 7.0)
    ctx.close()

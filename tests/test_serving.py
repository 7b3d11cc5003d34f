"""Continuous-batching server: results alone equal results in the mix,
admission under a memory budget, and a short Poisson stream whose every
request reports exactly its pulled-through pairs."""
import numpy as np
import pytest

import oracle
from paper_2106_12655_amd import serve

pytestmark = pytest.mark.gpu

SMALL = [("chainmail", 600, 32), ("knit", 500, 64), ("chainmail", 1500, 128), ("knit", 800, 256)]


def _pool(steps=2):
    pool = []
    for k, (kind, L, N) in enumerate(SMALL):
        base = serve.scene(kind, 100 + k, L, N)
        pool.append({"kind": kind, "base": base, "n_loops": base.n_loops, "nseg": N,
                     "steps": [serve.timestep(kind, base, 100 + k, L, N, s) for s in range(steps)]})
    return pool


def test_alone_equals_mix():
    import torch
    pool = _pool()
    srv = serve.Server(slots=4)
    sids = [srv.open_session(e["base"].offsets, e["base"].exp_pairs, e["base"].exp_lk) for e in pool]
    jobs = [(k, s) for k in range(len(pool)) for s in range(2)]
    dev = {(k, s): torch.from_numpy(pool[k]["steps"][s][0]).cuda() for k, s in jobs}
    alone = {}
    for k, s in jobs:
        alone[(k, s)] = srv.wait(srv.submit(sids[k], dev[(k, s)]), fetch=True, cap=400000)
    rids = {(k, s): srv.submit(sids[k], dev[(k, s)]) for k, s in jobs}
    mix = {j: srv.wait(r, fetch=True, cap=400000) for j, r in rids.items()}
    overlap = 0
    for j in jobs:
        a, m = alone[j], mix[j]
        assert a["status"] == 0 and m["status"] == 0
        assert np.array_equal(a["pairs"], m["pairs"])
        assert np.array_equal(a["lk"], m["lk"])
        assert np.array_equal(a["real"].view(np.int64), m["real"].view(np.int64)), j
        changed = {tuple(x) for x in pool[j[0]]["steps"][j[1]][1].tolist()}
        assert {(r[0], r[1]) for r in m["mismatches"].tolist()} == changed
        assert len(changed) > 0
        # the server's comparison against the oracle's, on the request's own matrix
        b = pool[j[0]]["base"]
        assert m["mismatches"].tolist() == oracle.verify(m["pairs"], m["lk"], b.exp_pairs,
                                                         b.exp_lk).tolist()
    starts = sorted((mix[j]["t_admit"], mix[j]["t_done"]) for j in jobs)
    for a, b in zip(starts, starts[1:]):
        overlap += b[0] < a[1]
    print("requests that started while another ran:", overlap, flush=True)
    assert overlap >= 1
    srv.close()


def test_admission_under_a_small_budget():
    import torch
    pool = _pool(steps=1)
    e = pool[2]
    b = e["base"]
    est = b.xyz.nbytes + 16 * b.n_loops * 40 + 16 * len(b.exp_pairs) + 4096
    srv = serve.Server(slots=4, budget=int(est * 1.2))
    sid = srv.open_session(b.offsets, b.exp_pairs, b.exp_lk)
    x = e["steps"][0][0]
    rids = [srv.submit(sid, x) for _ in range(4)]  # host memory: copied per request
    res = [srv.wait(r, fetch=True, cap=400000) for r in rids]
    for r in res:
        assert r["status"] == 0 and r["n_mismatch"] == len(e["steps"][0][1])
        assert np.array_equal(r["real"].view(np.int64), res[0]["real"].view(np.int64))
    # the budget admits one request at a time: runs do not overlap
    spans = sorted((r["t_admit"], r["t_done"]) for r in res)
    for a, c in zip(spans, spans[1:]):
        assert c[0] >= a[1] - 1e-6
    big = serve.scene("chainmail", 7, 20000, 256)
    sid2 = srv.open_session(big.offsets, big.exp_pairs, big.exp_lk)
    with pytest.raises(Exception):
        srv.submit(sid2, np.zeros((big.offsets[-1], 3), np.float32))
    srv.close()


def test_poisson_stream_reports_pulled_pairs():
    pool = _pool(steps=2)
    srv = serve.Server(slots=4)
    recs = serve.run_stream(srv, pool, rate=200.0, n_requests=24, seed=3)
    summ = serve.summarize(recs)
    print("stream:", summ, flush=True)
    assert summ["exact"] == 24
    assert summ["p99_ms"] >= summ["p50_ms"] > 0
    srv.close()


@pytest.mark.parametrize("mode", ["crossings", "barnes_hut", "plain"])
def test_stream_in_other_modes(mode):
    """The server runs any mode of the direct-sum call: every request of a
    short stream reports exactly its pulled-through pairs."""
    pool = _pool(steps=2)
    srv = serve.Server(slots=4, mode=mode)
    recs = serve.run_stream(srv, pool, rate=200.0, n_requests=16, seed=5)
    summ = serve.summarize(recs)
    print("stream (%s):" % mode, summ, flush=True)
    assert summ["exact"] == 16
    srv.close()


@pytest.mark.parametrize("mode", ["crossings", "barnes_hut"])
def test_sessions_come_and_go(mode):
    """Sessions opened and closed in turn (their resident offsets may reuse a
    closed session's device address): every request stays exact.  The budget
    (96 MiB) holds one request with the workspace its mode grows to (the
    Barnes-Hut lists of the largest scene are about 60 MB), so the second slot
    waits for it rather than allocate beside it."""
    pool = _pool(steps=1)
    srv = serve.Server(slots=2, mode=mode, budget=96 << 20)
    for rep in range(2):
        for e in pool:
            b = e["base"]
            sid = srv.open_session(b.offsets, b.exp_pairs, b.exp_lk)
            x, changed = e["steps"][0]
            r = srv.wait(srv.submit(sid, x), fetch=True, cap=400000)
            assert r["status"] == 0, (mode, rep, e["kind"])
            assert {(m[0], m[1]) for m in r["mismatches"].tolist()} == {tuple(c) for c in changed.tolist()}
            srv.close_session(sid)
    srv.close()

"""Continuous-batching verification service on one GPU (Python face of lk_server).

The native server (csrc/lk_server.hip) queues requests, admits them in
arrival order as slots and the device-memory budget free up, and runs them
concurrently; this module wraps it, builds the per-timestep workloads, and
drives a Poisson stream of requests to measure latency percentiles beside
throughput.

Workload of the stream: each request is one timestep of a perturbed
chainmail sheet or knit tube set with 500-20,000 loops of 32-4,096 segments
(log-uniform), per-vertex Gaussian noise (0.05 for chainmail, laid out on a
1.25 row pitch so that unlinked rings keep 0.4 apart; 0.01 for knit rows,
whose clasps are only ~0.13 apart), and about 1% of the linked (or, for knit,
clasped) pairs pulled through: edge rings slid out of the sheet, or knit
clasps reversed.  The session's expected matrix is the
unperturbed construction, so every request must report exactly its pulled
pairs as mismatches.

Run: ``python -m paper_2106_12655_amd.serve --requests 200 --load 0.7``.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import threading
import time

import numpy as np

from . import _lib
from . import inputs as I


class Server:
    """lk_server: `slots` concurrent requests, a device-memory budget in bytes
    (0 = 80% of free memory), one direct-sum mode for all requests."""

    def __init__(self, device=0, slots=4, budget=0, mode="mixed", max_loops=20000,
                 max_pairs=400000):
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        m = _lib.MODES[mode]
        st = self.lib.lk_server_create(ctypes.byref(h), int(device), int(slots), int(budget), m,
                                       int(max_loops), int(max_pairs))
        if st != _lib.OK:
            raise _lib.LkError(st, "lk_server_create failed")
        self.h = h
        self._keep = {}

    def _check(self, st):
        if st != _lib.OK:
            raise _lib.LkError(st, self.lib.lk_server_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.lk_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def open_session(self, offsets, exp_pairs, exp_lk) -> int:
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        ep = np.ascontiguousarray(np.asarray(exp_pairs, dtype=np.int32).reshape(-1, 2))
        el = np.ascontiguousarray(np.asarray(exp_lk, dtype=np.int32))
        sid = ctypes.c_int64(0)
        self._check(self.lib.lk_server_open_session(
            self.h, off.ctypes.data_as(ctypes.c_void_p), off.shape[0] - 1,
            ep.ctypes.data_as(ctypes.c_void_p), el.ctypes.data_as(ctypes.c_void_p), el.shape[0],
            ctypes.byref(sid)))
        return int(sid.value)

    def close_session(self, sid: int):
        self._check(self.lib.lk_server_close_session(self.h, int(sid)))

    def submit(self, sid: int, xyz) -> int:
        """xyz: numpy array (host) or torch tensor on the GPU (used in place).
        The array must stay alive until the request is waited for."""
        try:
            import torch
            is_dev = isinstance(xyz, torch.Tensor) and xyz.is_cuda
        except ImportError:
            is_dev = False
        if is_dev:
            ptr, where = ctypes.c_void_p(xyz.data_ptr()), _lib.MEM_DEVICE
            dt = _lib.F64 if xyz.dtype == torch.float64 else _lib.F32
        else:
            xyz = np.ascontiguousarray(xyz)
            ptr, where = xyz.ctypes.data_as(ctypes.c_void_p), _lib.MEM_HOST
            dt = _lib.F64 if xyz.dtype == np.float64 else _lib.F32
        rid = ctypes.c_int64(0)
        self._check(self.lib.lk_server_submit(self.h, int(sid), ptr, dt, where, ctypes.byref(rid)))
        self._keep[int(rid.value)] = xyz
        return int(rid.value)

    def wait(self, rid: int, timeout_ms: int = -1, fetch: bool = False, cap: int = 1 << 20):
        """Result dict of a request; with fetch=True also its pairs, integers,
        reals and mismatch records (numpy)."""
        res = _lib.Result()
        if fetch:
            pairs = np.zeros((cap, 2), np.int32)
            lk = np.zeros(cap, np.int32)
            real = np.zeros(cap, np.float64)
            mism = np.zeros((cap, 4), np.int32)
            args = [a.ctypes.data_as(ctypes.c_void_p) for a in (pairs, lk, real, mism)]
        else:
            args = [None, None, None, None]
        st = self.lib.lk_server_wait(self.h, int(rid), int(timeout_ms), ctypes.byref(res), *args,
                                     int(cap) if fetch else 0)
        self._check(st)
        self._keep.pop(int(rid), None)
        out = {k: getattr(res, k) for k, _ in res._fields_}
        if fetch:
            n = min(out["n_pairs"], cap)
            out.update(pairs=pairs[:n], lk=lk[:n], real=real[:n],
                       mismatches=mism[:min(out["n_mismatch"], cap)])
        return out


# --------------------------------------------------------------- workloads
def scene(kind: str, seed: int, n_loops: int, nseg: int):
    """Structure of one simulated object: a chainmail sheet of about n_loops
    rings of nseg segments, or knit tubes of about n_loops rows of about nseg
    segments each.  Returns the unperturbed LoopSet (the certificate)."""
    if kind == "chainmail":
        cols = max(2, int(round(np.sqrt(n_loops * 1.4))))
        rows = max(2, n_loops // cols)
        return I.chainmail(seed, rows=rows, cols=cols, nseg=nseg, sigma=0.0, row_pitch=1.25)
    cp = int(np.clip(nseg // 8, 16, 128))
    cp -= cp % 8
    per_span = max(1, nseg // cp)
    return I.knit(seed, n_loops=n_loops, cp_min=cp, cp_max=cp, per_span=per_span,
                  linked_fraction=0.0)


def timestep(kind: str, base, seed: int, n_loops: int, nseg: int, step: int,
             pull_frac: float = 0.01):
    """One perturbed timestep of a scene: per-vertex noise and ~pull_frac of
    its linked (chainmail) or clasped (knit) pairs pulled through.  Returns
    (xyz float32, the pairs whose value must differ from the certificate)."""
    rng = np.random.default_rng([seed, step])
    if kind == "chainmail":
        cols = max(2, int(round(np.sqrt(n_loops * 1.4))))
        rows = max(2, n_loops // cols)
        edge = np.concatenate([np.arange(cols), (rows - 1) * cols + np.arange(cols)])
        k = int(min(len(edge), max(1, round(pull_frac * len(base.exp_pairs) / 2))))
        rings = rng.choice(edge, size=k, replace=False)
        ls = I.chainmail(seed, rows=rows, cols=cols, nseg=nseg, sigma=0.05, row_pitch=1.25,
                         pulled_rings=rings.tolist(), noise_seed=int(rng.integers(1 << 31)))
        changed = ls.meta["pulled"]
    else:
        cp = int(np.clip(nseg // 8, 16, 128))
        cp -= cp % 8
        per_span = max(1, nseg // cp)
        starts = set(base.meta["row_starts"])
        cand = np.array([r for r in range(1, base.n_loops) if r not in starts])
        k = max(1, int(round(pull_frac * len(cand))))
        pull = rng.choice(cand, size=k, replace=False)
        ls = I.knit(seed, n_loops=n_loops, cp_min=cp, cp_max=cp, per_span=per_span,
                    linked_fraction=0.0, sigma=0.01, pull=pull.tolist(),
                    noise_seed=int(rng.integers(1 << 31)))
        changed = np.array(sorted([[int(r) - 1, int(r)] for r in pull]), np.int32).reshape(-1, 2)
    return ls.xyz.astype(np.float32), changed


def make_pool(seed: int, n_scenes: int, steps_per_scene: int = 1, l_range=(500, 20000),
              n_range=(32, 4096), max_terms: float | None = None):
    """Scenes with log-uniform sizes and a few perturbed timesteps each."""
    rng = np.random.default_rng(seed)
    pool = []
    for k in range(n_scenes):
        kind = "chainmail" if k % 2 == 0 else "knit"
        L = int(np.exp(rng.uniform(np.log(l_range[0]), np.log(l_range[1]))))
        N = int(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))
        if max_terms is not None:
            while 5.0 * L * N * N > max_terms and N > n_range[0]:
                N = max(n_range[0], N // 2)
        base = scene(kind, seed * 1000 + k, L, N)
        steps = [timestep(kind, base, seed * 1000 + k, L, N, s) for s in range(steps_per_scene)]
        pool.append({"kind": kind, "n_loops": base.n_loops, "nseg": N, "base": base,
                     "steps": steps})
    return pool


def run_stream(server: Server, pool, rate: float, n_requests: int, seed: int = 0,
               device_resident: bool = True):
    """Submit n_requests Poisson arrivals (rate per second) drawn from the
    pool; returns per-request records (latency = done - submit)."""
    import torch
    rng = np.random.default_rng(seed)
    sessions = []
    for e in pool:
        b = e["base"]
        sid = server.open_session(b.offsets, b.exp_pairs, b.exp_lk)
        dev = [torch.from_numpy(x).cuda() if device_resident else x for x, _ in e["steps"]]
        sessions.append((sid, dev))
    torch.cuda.synchronize()
    picks = rng.integers(0, len(pool), size=n_requests)
    steps = [int(rng.integers(0, len(pool[p]["steps"]))) for p in picks]
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    ids, records = [], [None] * n_requests
    lock = threading.Lock()

    def waiter():
        for k in range(n_requests):
            while True:
                with lock:
                    if k < len(ids):
                        rid = ids[k]
                        break
                time.sleep(0.0005)
            r = server.wait(rid, fetch=True, cap=400000)
            p, s = picks[k], steps[k]
            changed = pool[p]["steps"][s][1]
            got = {(int(a), int(b)) for a, b, _, _ in r["mismatches"]}
            want = {(int(a), int(b)) for a, b in changed}
            records[k] = {"scene": int(p), "kind": pool[p]["kind"], "loops": pool[p]["n_loops"],
                          "nseg": pool[p]["nseg"], "latency": r["t_done"] - r["t_submit"],
                          "queue": r["t_admit"] - r["t_submit"],
                          "service": r["t_done"] - r["t_admit"], "terms": r["terms"],
                          "pairs": r["n_pairs"], "mismatch": r["n_mismatch"],
                          "exact": got == want and r["status"] == 0, "status": r["status"],
                          "t_submit": r["t_submit"], "t_done": r["t_done"],
                          "refits": r["refits"], "flagged": r["n_flagged"]}

    th = threading.Thread(target=waiter)
    th.start()
    t_next = time.perf_counter()
    for k in range(n_requests):
        t_next += gaps[k]
        dt = t_next - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        sid, dev = sessions[picks[k]]
        rid = server.submit(sid, dev[steps[k]])
        with lock:
            ids.append(rid)
    th.join()
    for sid, _ in sessions:
        server.close_session(sid)
    return records


def _pct(v, q):
    return float(np.percentile(v, q) * 1e3) if len(v) else 0.0


def summarize(records, alone=None):
    """Latency percentiles beside throughput.  With `alone` (each scene's
    service time when it runs by itself), also the slowdown of every request
    (latency / alone) and, per size class of that alone time, the split of
    latency into queueing (submit to admission) and service (admission to
    results on the host)."""
    lat = np.array([r["latency"] for r in records])
    terms = np.array([r["terms"] for r in records])
    span = max(r["t_done"] for r in records) - min(r["t_submit"] for r in records)
    out = {"requests": len(records), "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
           "mean_ms": float(lat.mean() * 1e3),
           "queue_p50_ms": _pct([r["queue"] for r in records], 50),
           "queue_p99_ms": _pct([r["queue"] for r in records], 99),
           "throughput_req_s": len(records) / span, "terms_per_s": float(terms.sum() / span),
           "exact": int(sum(r["exact"] for r in records)),
           "refits": int(sum(r["refits"] for r in records)), "span_s": span}
    if alone is not None:
        slow = np.array([r["latency"] / alone[r["scene"]] for r in records])
        out["slowdown_p50"] = float(np.percentile(slow, 50))
        out["slowdown_p99"] = float(np.percentile(slow, 99))
        classes = {}
        for name, lo, hi in (("alone<10ms", 0.0, 0.01), ("alone 10-100ms", 0.01, 0.1),
                             ("alone>=100ms", 0.1, np.inf)):
            rs = [r for r in records if lo <= alone[r["scene"]] < hi]
            if not rs:
                continue
            classes[name] = {
                "requests": len(rs),
                "latency_p50_ms": _pct([r["latency"] for r in rs], 50),
                "latency_p99_ms": _pct([r["latency"] for r in rs], 99),
                "queue_p50_ms": _pct([r["queue"] for r in rs], 50),
                "queue_p99_ms": _pct([r["queue"] for r in rs], 99),
                "service_p50_ms": _pct([r["service"] for r in rs], 50),
                "service_p99_ms": _pct([r["service"] for r in rs], 99),
            }
        out["by_class"] = classes
    return out


def service_times(server: Server, pool) -> list:
    """Each pool entry's service time (admission to results on the host)
    when it runs alone on the server."""
    import torch
    out = []
    for e in pool:
        b = e["base"]
        sid = server.open_session(b.offsets, b.exp_pairs, b.exp_lk)
        x = torch.from_numpy(e["steps"][0][0]).cuda()
        r = server.wait(server.submit(sid, x))
        out.append(r["t_done"] - r["t_admit"])
        server.close_session(sid)
    return out


def capacity(server: Server, pool) -> float:
    """Requests per second the server sustains when each pool entry is run
    alone, back to back (the service rate the offered load is scaled to)."""
    return len(pool) / sum(service_times(server, pool))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--load", type=float, default=0.7)
    ap.add_argument("--scenes", type=int, default=12)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-terms", type=float, default=2e11)
    args = ap.parse_args()
    pool = make_pool(args.seed, args.scenes, max_terms=args.max_terms)
    srv = Server(slots=args.slots)
    cap = capacity(srv, pool)
    recs = run_stream(srv, pool, args.load * cap, args.requests, args.seed)
    out = summarize(recs)
    out.update(capacity_req_s=cap, load=args.load, slots=args.slots)
    print(json.dumps(out))
    srv.close()


if __name__ == "__main__":
    main()

"""Throughput of the direct-summation linking-number path on one MI355X.

A step is one full lk_direct_sum over every candidate pair of the workload:
loop validation, planning, the persistent Eq. 4 kernel, rounding/flagging and
(MIXED) the FP64 refit of ambiguous pairs.  Geometry, offsets and the pair
list are resident in HBM before the timed region; the potential link search
runs once before it (reported separately, like the paper's PLS column).  The
timed steps are the library's default launch path (the call's kernel sequence
captured once into a HIP graph and replayed); an equal number of eager calls
with HIP events around the main kernel gives its time for the roofline.

Default workload: the 4-in-1 chainmail sheet (14,000 rings x 64 segments,
FP32, ~69k candidate pairs, 2.8e8 segment-pair terms) in the mixed-precision
mode; the plain FP64 mode is timed on the same input and reported beside it.

Before timing, the library's autotuner picks the kernel configuration for
the workload (on a seeded subset of pairs for the two largest workloads).

The default run adds two companion objects: ``knit`` (the knit-like
workload, 2,000 B-spline rows of 512-16,128 segments, mixed and plain, each
with its roofline fraction) and ``serving`` (a Poisson stream of 1,000
verification requests against the continuous-batching server at 0.7 of its
capacity: throughput, p50/p99 latency, queueing and service per size class).
``--config serving`` makes the stream the headline instead.

Prints ONE JSON line.  Options:
  --steps K --warmup W   timed / untimed steps (default 20 / 3)
  --config NAME          ring_grid | chainmail | knit | long_pairs | serving
  --mode mixed|plain|crossings|barnes_hut
                         mode of the headline value (default mixed); with mixed,
                         plain FP64, the crossing count (Alg. 4) and Barnes-Hut
                         (Alg. 6: beta 4, and the adaptive beta from 2) are timed
                         on the same input and reported beside it
  --no-plain, --no-crossings, --no-bh, --no-dz, --no-knit, --no-serving
                         skip those companion legs
                         (dz: the discretization of Alg. 3, timed on the knit
                         workload's B-spline control points, 314k spans)
  --dz-only              only the discretization leg (profiling)
  --no-cpu-baseline      skip the oracle leg
  --no-tune              keep the default kernel configuration
  --gpus N               only N = 1 is supported (one GPU per process)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_TERM = 90  # arithmetic of Eq. 4 as printed in Alg. 5 (sqrt/atan2 not counted)
# crossing count: a 2D segment-intersection test is four orientation
# determinants of 5 FLOP each (projection and sign bookkeeping not counted)
FLOP_PER_TERM_CC = 20
PEAK_FP32_TFLOPS = 157.3  # MI355X published FP32 vector peak
PEAK_FP64_TFLOPS = 78.6   # MI355X published FP64 vector peak

# HBM bytes per launch of the direct-sum kernel, from two rocprofv3 --pmc runs
# of the chainmail command (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch,
# averaged over the kernel's dispatches), each scaled by what the same counter
# read for one 256 MiB elementwise copy in that run (fetch x2.000, write
# x1.000), for the launch configuration the autotuner picked.  A record only
# holds for the machine code it was taken on (the fingerprint of the kernel's
# gfx950 assembly that the build writes to liblk.kernels.json) and for its
# launch configuration: anything else reports traffic as null.
TRAFFIC = {
    ("chainmail", "mixed"): {
        "kernel": "_ZN2lk12_GLOBAL__N_113ds_persistentIffLi2ELi4ELb1EEEvNS_6DsArgsE",
        "isa": "69e07da7d58f865f",
        "config": {"segs_per_lane": 4, "tile_a": 512, "chunk_a": 4096, "atan_form": 2},
        "fetch_scale": 2.000, "write_scale": 1.000,
        # (effective small batch, waves_per_cu) -> (FETCH_SIZE, WRITE_SIZE) KiB
        # per launch.  The runtime raises a batch below segs_per_lane to it,
        # so batches 1, 2 and 4 launch the same work here.
        "by_launch": {(4, 0): (24062.6, 2578.0), (4, 8): (24043.7, 2561.1),
                      (4, 12): (23789.7, 2563.9), (8, 0): (21175.3, 1963.6),
                      (8, 8): (21215.4, 1951.1), (8, 12): (21192.9, 1959.5),
                      (16, 0): (19740.0, 1598.0), (16, 8): (19742.0, 1605.9),
                      (16, 12): (19707.8, 1608.5)},
        "source": "profiles/ds_persistent_chainmail_hbm_traffic.txt",
    },
}


WORKLOADS = {
    "ring_grid": "64 rings x 32 segments on an 8x8 grid, FP64, 105 candidate pairs",
    "chainmail": "4-in-1 chainmail, 14,000 rings x 64 segments, FP32",
    "knit": "knit-like tubes, 2,000 B-spline rows of 512-16,384 segments, FP32",
    "long_pairs": "16 pairs of long winding loops, 2^18-2^20 segments each, FP32",
    "serving": "Poisson stream of chainmail/knit timesteps, 500-20,000 loops x 32-4,096 segments",
}


_T0 = time.perf_counter()


def log(msg: str):
    """One progress line on stderr as each leg ends (the JSON line is stdout)."""
    print("bench %6.1fs: %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


def kernel_isa(symbol: str):
    """Fingerprint of a kernel's assembly in the built library, or None."""
    try:
        with open(os.path.join(ROOT, "paper_2106_12655_amd", "liblk.kernels.json")) as fh:
            return json.load(fh)["kernels"].get(symbol)
    except (OSError, ValueError, KeyError):
        return None


def measured_traffic(config: str, mode: str, tuned):
    """HBM bytes per launch from the recorded counters, or None when the record
    does not match the kernel's machine code or the launch configuration."""
    rec = TRAFFIC.get((config, mode))
    if rec is None or tuned is None or kernel_isa(rec["kernel"]) != rec["isa"]:
        return None
    if any(tuned.get(k) != v for k, v in rec["config"].items()):
        return None
    batch = max(tuned.get("small_batch") or 0, tuned.get("segs_per_lane") or 0)
    kib = rec["by_launch"].get((batch, tuned.get("waves_per_cu")))
    if kib is None:
        return None
    return (kib[0] * rec["fetch_scale"] + kib[1] * rec["write_scale"]) * 1024


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="chainmail", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="mixed", choices=["mixed", "plain", "crossings", "barnes_hut"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-FP64 companion run")
    ap.add_argument("--no-crossings", action="store_true",
                    help="skip the crossing-count companion run")
    ap.add_argument("--no-bh", action="store_true", help="skip the Barnes-Hut companion run")
    ap.add_argument("--no-dz", action="store_true",
                    help="skip the discretization companion run (knit B-spline rows)")
    ap.add_argument("--dz-only", action="store_true",
                    help="time only the discretization leg (for profiling it)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: reuse a stored choice instead of searching")
    ap.add_argument("--no-knit", action="store_true",
                    help="skip the knit companion run (mixed and plain on the knit workload)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving companion run (Poisson stream of verification requests)")
    ap.add_argument("--serving-requests", type=int, default=1000,
                    help="requests in the serving companion's stream")
    ap.add_argument("--requests", type=int, default=200, help="serving: requests in the stream")
    ap.add_argument("--load", type=float, default=0.7, help="serving: offered load / capacity")
    ap.add_argument("--scenes", type=int, default=12, help="serving: distinct objects")
    return ap.parse_args()


def tune(ctx, ls, xyz, off, pairs, mode, lkmod, cache=None):
    """Autotune on the workload, or on a seeded subset of its pairs when a
    single call would take seconds (knit, long pairs)."""
    import torch
    pr = pairs.cpu().numpy()
    cost = ls.sizes[pr[:, 0]].astype(np.int64) * ls.sizes[pr[:, 1]]
    if cost.sum() > 5e10:
        rng = np.random.default_rng(0)
        order = rng.permutation(len(pr))
        keep = np.sort(order[np.cumsum(cost[order]) <= 5e10])
        if len(keep) == 0:
            keep = np.array([int(np.argmin(cost))])
        sub = torch.from_numpy(np.ascontiguousarray(pr[keep])).cuda()
    else:
        sub = pairs
    t0 = time.perf_counter()
    t = ctx.autotune(xyz, off, sub, mode, cache_path=cache)
    t["seconds"] = time.perf_counter() - t0
    t["pairs_used"] = int(sub.shape[0])
    return t


def time_mode(ctx, xyz, off, pairs, mode, steps, warmup, lkmod):
    """The timed region replays the call the way the library runs it by
    default (the first call on a stream is captured into a HIP graph, later
    identical calls replay it), bracketed by device synchronisation.  A second
    pass of the same number of eager calls, with the library's HIP-event ring
    around the main kernel (same stream), gives that kernel's time."""
    import torch
    out = ctx.direct_sum(xyz, off, pairs, mode)
    for _ in range(warmup):
        ctx.direct_sum(xyz, off, pairs, mode, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.direct_sum(xyz, off, pairs, mode, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    graph_replayed = bool(ctx.stats()["graph_replayed"])
    ctx.set_option(lkmod._lib.OPT_TIMING, max(steps, 1))
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    for _ in range(steps):
        ctx.direct_sum(xyz, off, pairs, mode, out=out)
    torch.cuda.synchronize()
    e1 = time.perf_counter()
    st = ctx.stats()
    ctx.set_option(lkmod._lib.OPT_TIMING, 0)
    real, lk, flags = [t.cpu().numpy() for t in out]
    return {
        "ms_per_step": (t1 - t0) * 1e3 / steps,
        "graph_replayed": graph_replayed,
        "eager_ms_per_step": (e1 - e0) * 1e3 / steps,
        "kernel_ms": st["kernel_ms"],
        "refit_kernel_ms": st["refit_kernel_ms"],
        "refits": int(np.sum(flags.view(np.uint32) & 1)),
        "refits_direct_sum": int(st.get("refits_direct_sum", 0)),
        "bh_reruns": int(st.get("bh_reruns", 0)),
        "real": real,
        "lk": lk,
        "flags": flags.view(np.uint32),
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2106_12655_amd as lk
    from paper_2106_12655_amd import inputs

    if args.config == "serving":
        return run_serving(args)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()  # a real stream: the null stream cannot be captured
    torch.cuda.set_stream(stream)
    if args.copy_probe_mib > 0:
        # one plain elementwise kernel that reads and writes exactly this many
        # bytes (dst = src * 1; a same-type copy_ would go to the DMA engine,
        # which the kernel counters do not see), so that profiler byte
        # counters can be scaled against a known transfer
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    ctx = lk.Context(0)
    if args.dz_only:
        line = {"discretization": time_discretize(ctx, args, lk, inputs)}
        ctx.close()
        print(json.dumps(line), flush=True)
        return
    ls = inputs.config(args.config, args.seed)
    xyz = torch.from_numpy(ls.xyz).cuda()
    off = torch.from_numpy(ls.offsets).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if ls.pairs is not None:
        pairs = torch.from_numpy(ls.pairs).cuda()
    else:
        pairs = ctx.build_pairs(xyz, off)
    torch.cuda.synchronize()
    pls_ms = (time.perf_counter() - t0) * 1e3
    pls_warm_ms = None
    if ls.pairs is None:  # again, with the search's buffers already allocated
        t0 = time.perf_counter()
        again = ctx.build_pairs(xyz, off)
        torch.cuda.synchronize()
        pls_warm_ms = (time.perf_counter() - t0) * 1e3
        assert torch.equal(again, pairs)
        del again
    pr = pairs.cpu().numpy()
    sizes = ls.sizes
    T = int(np.sum(sizes[pr[:, 0]].astype(np.int64) * sizes[pr[:, 1]]))
    exp = ls.expected_for(pr)

    # (Barnes-Hut has no tuned launch parameters)
    tuned = None if args.no_tune or args.mode == "barnes_hut" else tune(
        ctx, ls, xyz, off, pairs, args.mode, lk, args.tune_cache)
    res = time_mode(ctx, xyz, off, pairs, args.mode, args.steps, args.warmup, lk)
    log("%s %s: %.3f ms per step" % (args.config, args.mode, res["ms_per_step"]))
    other, tuned_plain = None, None
    if not args.no_plain and args.mode == "mixed":
        tuned_plain = None if args.no_tune else tune(ctx, ls, xyz, off, pairs, "plain", lk,
                                                     args.tune_cache)
        other = time_mode(ctx, xyz, off, pairs, "plain", max(args.steps // 2, 1),
                          min(args.warmup, 1), lk)
        log("plain: %.3f ms per step" % other["ms_per_step"])
    bh, bha = None, None
    if not args.no_bh and args.mode == "mixed":
        bh = time_mode(ctx, xyz, off, pairs, "barnes_hut", args.steps, args.warmup, lk)
        # the adaptive beta of Sec. 3.4.4 with the paper's CPU settings
        ctx.set_option(lk._lib.OPT_BH_BETA_MILLI, 2000)
        ctx.set_option(lk._lib.OPT_BH_ADAPTIVE, 1)
        bha = time_mode(ctx, xyz, off, pairs, "barnes_hut", args.steps, args.warmup, lk)
        ctx.set_option(lk._lib.OPT_BH_ADAPTIVE, 0)
        ctx.set_option(lk._lib.OPT_BH_BETA_MILLI, 4000)
        log("barnes_hut: %.3f ms per step" % bh["ms_per_step"])
    cc, tuned_cc = None, None
    if not args.no_crossings and args.mode == "mixed":
        tuned_cc = None if args.no_tune else tune(ctx, ls, xyz, off, pairs, "crossings", lk,
                                                  args.tune_cache)
        cc = time_mode(ctx, xyz, off, pairs, "crossings", args.steps, args.warmup, lk)
        if T <= 1e12:
            # the same count with culling off: every segment pair is tested, so
            # the kernel time prices the per-term work against the roofline
            ctx.set_option(lk._lib.OPT_CROSSING_CULL, 0)
            cc["exhaustive"] = time_mode(ctx, xyz, off, pairs, "crossings",
                                         max(min(args.steps, 5), 1), min(args.warmup, 1), lk)
            ctx.set_option(lk._lib.OPT_CROSSING_CULL, 1)
        log("crossings: %.3f ms per step" % cc["ms_per_step"])

    value = T / (res["ms_per_step"] * 1e-3)
    fp64 = args.mode == "plain"
    peak = PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS
    fpt = FLOP_PER_TERM_CC if args.mode == "crossings" else FLOP_PER_TERM  # (BH: covered pairs)
    achieved = fpt * T / (res["kernel_ms"] * 1e-3) / 1e12 if res["kernel_ms"] > 0 else 0.0
    line = {
        "metric": "segment-pair evals/s",
        "value": value,
        "unit": "segment-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else ("f32 predicates+f64" if args.mode == "crossings"
                                     else "f32+f64"),
        "data": "synthetic",
        "config": {"workload": args.config, "description": WORKLOADS[args.config],
                   "loops": int(ls.n_loops), "pairs": int(len(pr)), "terms": T,
                   "mode": args.mode, "seed": args.seed},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(args.config, args.mode, tuned),
                     "traffic_source": (TRAFFIC[(args.config, args.mode)]["source"]
                                        if measured_traffic(args.config, args.mode, tuned)
                                        is not None else None),
                     "kernel": "ds_persistent (%s)" % ("FP64" if fp64 else (
                         "FP32 crossing count" if args.mode == "crossings" else "FP32 terms")),
                     "kernel_ms": res["kernel_ms"], "flop_per_term": fpt},
        "graph_replayed": res["graph_replayed"],
        "eager_ms_per_step": res["eager_ms_per_step"],
        "tuned": tuned,
        "pls_ms": pls_ms,
        "pls_warm_ms": pls_warm_ms,
        "refits": res["refits"],
        "int_mismatch_vs_construction": int(np.sum(res["lk"] != exp)),
    }
    if other is not None:
        line["plain_f64"] = {
            "value": T / (other["ms_per_step"] * 1e-3),
            "ms_per_step": other["ms_per_step"],
            "eager_ms_per_step": other["eager_ms_per_step"],
            "kernel_ms": other["kernel_ms"],
            "roofline_frac_fp64": (FLOP_PER_TERM * T / (other["kernel_ms"] * 1e-3) / 1e12
                                   / PEAK_FP64_TFLOPS) if other["kernel_ms"] > 0 else 0.0,
            "int_mismatch_vs_mixed": int(np.sum(other["lk"] != res["lk"])),
            "max_abs_diff_vs_mixed": float(np.max(np.abs(other["real"] - res["real"]))),
            "tuned": tuned_plain,
        }
    if cc is not None:
        # value: segment pairs covered per second (culling skips most of them);
        # the roofline fraction comes from the exhaustive run, which tests all
        line["crossings"] = {
            "value": T / (cc["ms_per_step"] * 1e-3),
            "ms_per_step": cc["ms_per_step"],
            "eager_ms_per_step": cc["eager_ms_per_step"],
            "kernel_ms": cc["kernel_ms"],
            "refit_kernel_ms": cc["refit_kernel_ms"],
            "refits": cc["refits"],
            "refits_direct_sum": cc["refits_direct_sum"],
            "int_mismatch_vs_mixed": int(np.sum(cc["lk"] != res["lk"])),
            "int_mismatch_vs_construction": int(np.sum(cc["lk"] != exp)),
            "tuned": tuned_cc,
        }
        ex = cc.get("exhaustive")
        if ex is not None:
            ach = FLOP_PER_TERM_CC * T / (ex["kernel_ms"] * 1e-3) / 1e12 if ex["kernel_ms"] > 0 else 0.0
            line["crossings"]["exhaustive"] = {
                "value": T / (ex["ms_per_step"] * 1e-3),
                "ms_per_step": ex["ms_per_step"],
                "kernel_ms": ex["kernel_ms"],
                "roofline_frac_fp32": ach / PEAK_FP32_TFLOPS,
                "flop_per_term": FLOP_PER_TERM_CC,
                "int_mismatch_vs_culled": int(np.sum(ex["lk"] != cc["lk"])),
            }
    if bh is not None:
        line["barnes_hut"] = {
            "value": T / (bh["ms_per_step"] * 1e-3),
            "ms_per_step": bh["ms_per_step"],
            "eager_ms_per_step": bh["eager_ms_per_step"],
            "kernel_ms": bh["kernel_ms"],
            "refit_kernel_ms": bh["refit_kernel_ms"],
            "refits": bh["refits"],
            "beta": 4.0, "order": 2,
            "max_abs_diff_vs_mixed": float(np.max(np.abs(bh["real"] - res["real"]))) if len(pr) else 0.0,
            "int_mismatch_vs_mixed": int(np.sum(bh["lk"] != res["lk"])),
            "int_mismatch_vs_construction": int(np.sum(bh["lk"] != exp)),
        }
        if bha is not None:
            line["barnes_hut"]["adaptive"] = {
                "beta_init": 2.0, "beta_max": 10.0, "target": 0.2,
                "value": T / (bha["ms_per_step"] * 1e-3),
                "ms_per_step": bha["ms_per_step"],
                "kernel_ms": bha["kernel_ms"],
                "pairs_evaluated_again": bha["bh_reruns"],
                "refits": bha["refits"],
                "max_abs_diff_vs_mixed": float(np.max(np.abs(bha["real"] - res["real"]))) if len(pr) else 0.0,
                "int_mismatch_vs_construction": int(np.sum(bha["lk"] != exp)),
            }
    if not args.no_cpu_baseline:
        line["cpu_baseline"], errs = cpu_baseline(ls, pr, res, other, args.cpu_threads, cc)
        line.update(errs)
        log("oracle baseline: %.1f s" % line["cpu_baseline"]["seconds"])
    if not args.no_dz:
        line["discretization"] = time_discretize(ctx, args, lk, inputs)
        log("discretization: %.3f ms per call" % line["discretization"]["ms_per_call"])
    ctx.close()
    if args.mode == "mixed" and args.config == "chainmail":
        if not args.no_knit:
            line["knit"] = knit_leg(args, lk, inputs)
            log("knit: mixed %.1f ms, plain %.1f ms per step" % (
                line["knit"]["mixed"]["ms_per_step"], line["knit"]["plain"]["ms_per_step"]))
        if not args.no_serving:
            line["serving"] = serving_leg(args, args.serving_requests, args.load, args.scenes,
                                          "mixed")
            log("serving: p50 %.1f ms, p99 %.1f ms" % (line["serving"]["latency"]["p50_ms"],
                                                       line["serving"]["latency"]["p99_ms"]))
    print(json.dumps(line), flush=True)


def knit_leg(args, lk, inputs):
    """The knit-like workload (2,000 closed B-spline rows of 512-16,128
    segments, 6,324 candidate pairs, 5.0e11 terms, FP32) on a context of its
    own: mixed and plain FP64, each autotuned on a seeded subset of the pairs,
    timed like the headline (graph replays, then eager calls with the main
    kernel's HIP events)."""
    import torch
    ls = inputs.config("knit", args.seed)
    ctx = lk.Context(0)
    xyz = torch.from_numpy(ls.xyz).cuda()
    off = torch.from_numpy(ls.offsets).cuda()
    pairs = ctx.build_pairs(xyz, off)
    pr = pairs.cpu().numpy()
    T = int(np.sum(ls.sizes[pr[:, 0]].astype(np.int64) * ls.sizes[pr[:, 1]]))
    exp = ls.expected_for(pr)
    out = {"workload": "knit", "description": WORKLOADS["knit"], "loops": int(ls.n_loops),
           "pairs": int(len(pr)), "terms": T, "seed": args.seed}
    legs = {}
    for mode, steps in (("mixed", 3), ("plain", 2)):
        tuned = None if args.no_tune else tune(ctx, ls, xyz, off, pairs, mode, lk, args.tune_cache)
        r = time_mode(ctx, xyz, off, pairs, mode, steps, 1, lk)
        peak = PEAK_FP64_TFLOPS if mode == "plain" else PEAK_FP32_TFLOPS
        ach = FLOP_PER_TERM * T / (r["kernel_ms"] * 1e-3) / 1e12 if r["kernel_ms"] > 0 else 0.0
        legs[mode] = r
        out[mode] = {"value": T / (r["ms_per_step"] * 1e-3), "unit": "segment-pairs/s",
                     "ms_per_step": r["ms_per_step"], "steps": steps,
                     "graph_replayed": r["graph_replayed"],
                     "eager_ms_per_step": r["eager_ms_per_step"], "kernel_ms": r["kernel_ms"],
                     "roofline": {"bound": "alu", "achieved": ach, "peak": peak,
                                  "unit": "TFLOP/s", "frac": ach / peak},
                     "refits": r["refits"],
                     "int_mismatch_vs_construction": int(np.sum(r["lk"] != exp)),
                     "tuned": tuned}
    out["mixed"]["max_abs_diff_vs_plain"] = float(np.max(np.abs(legs["mixed"]["real"] -
                                                               legs["plain"]["real"])))
    out["mixed"]["int_mismatch_vs_plain"] = int(np.sum(legs["mixed"]["lk"] != legs["plain"]["lk"]))
    ctx.close()
    return out


def serving_leg(args, n_requests, load, scenes, mode):
    """A Poisson stream of verification requests against the continuous-
    batching server (4 slots): chainmail and knit timesteps of 500-20,000
    loops x 32-4,096 segments (at most 3e11 terms each), at `load` times the
    rate the server sustains when each scene runs alone back to back.
    Latency is submit to results on the host; it is split into queueing and
    service per size class, and each request's slowdown over its scene's
    time alone is reported."""
    import torch
    from paper_2106_12655_amd import serve
    t0 = time.perf_counter()
    pool = serve.make_pool(args.seed, scenes, max_terms=3e11)
    gen_s = time.perf_counter() - t0
    srv = serve.Server(slots=4, mode=mode)
    log("serving: %d scenes built in %.1f s" % (len(pool), gen_s))
    alone = serve.service_times(srv, pool)
    cap = len(pool) / sum(alone)
    log("serving: capacity %.1f requests/s alone; stream of %d at load %.2f" % (
        cap, n_requests, load))
    recs = serve.run_stream(srv, pool, load * cap, n_requests, args.seed)
    summ = serve.summarize(recs, alone)
    srv.close()
    torch.cuda.synchronize()
    return {
        "workload": "serving", "description": WORKLOADS["serving"], "mode": mode,
        "requests": n_requests, "load": load, "scenes": scenes, "slots": 4,
        "value": summ["terms_per_s"], "unit": "segment-pairs/s",
        "latency": {"p50_ms": summ["p50_ms"], "p99_ms": summ["p99_ms"],
                    "mean_ms": summ["mean_ms"], "queue_p50_ms": summ["queue_p50_ms"],
                    "queue_p99_ms": summ["queue_p99_ms"],
                    "slowdown_p50": summ["slowdown_p50"], "slowdown_p99": summ["slowdown_p99"]},
        "by_class": summ["by_class"],
        "throughput_req_s": summ["throughput_req_s"], "capacity_req_s": cap,
        "span_s": summ["span_s"], "requests_exact": summ["exact"], "refits": summ["refits"],
        "pool_seconds": gen_s,
        "pool": [{"kind": e["kind"], "loops": e["n_loops"], "nseg": e["nseg"],
                  "alone_ms": a * 1e3, "changed": int(len(e["steps"][0][1]))}
                 for e, a in zip(pool, alone)],
    }


def time_discretize(ctx, args, lk, inputs):
    """Alg. 3 on the knit workload's control polygons (2,000 closed uniform
    cubic B-spline rows, 314k spans): wall time per lk_discretize call (it
    synchronises once per pass), the output size, and the linking numbers of
    the output polylines (MIXED direct sum) against the construction's.  The
    oracle's discretization is timed on a bounded sample: the first rows of
    the same workload."""
    import torch
    import oracle
    k = inputs.knit(args.seed, per_span=0, dtype=np.float64)
    x = torch.from_numpy(k.xyz).cuda()
    o = torch.from_numpy(k.offsets).cuda()
    pr = ctx.build_pairs(x, o)
    cap = 4 * len(k.xyz) + 1024
    for _ in range(max(args.warmup, 1)):
        out = ctx.discretize(x, o, pr, "bspline", cap)
    torch.cuda.synchronize()
    steps = max(args.steps, 1)
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.discretize(x, o, pr, "bspline", cap)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    xyz, off, flags, info = out
    _, lk_int, _ = ctx.direct_sum(xyz, off, pr, "mixed")
    pairs = pr.cpu().numpy()
    exp = k.expected_for(pairs)
    got = lk_int.cpu().numpy()
    # the polyline through the knots (one vertex per span) for contrast
    knots = torch.from_numpy(inputs.knit(args.seed, per_span=1, dtype=np.float64).xyz).cuda()
    _, lk_knots, _ = ctx.direct_sum(knots, o, pr, "mixed")
    leg = {
        "workload": "knit control polygons: %d closed B-spline rows, %d spans, %d pairs" % (
            k.n_loops, len(k.xyz), len(pairs)),
        "value": len(k.xyz) / (ms * 1e-3), "unit": "input spans/s", "ms_per_call": ms,
        "steps": steps, "passes": info["passes"], "input_spans": info["input_spans"],
        "vertices": info["vertices"], "splits": info["splits"],
        "loops_flagged": int((flags.cpu().numpy() != 0).sum()),
        "int_mismatch_vs_construction": int(np.sum(got != exp)),
        "knot_polyline_int_mismatch_vs_construction": int(np.sum(lk_knots.cpu().numpy() != exp)),
        "linked_pairs": int(np.sum(exp != 0)),
    }
    if not args.no_cpu_baseline:
        sub = inputs.knit(args.seed, n_loops=150, per_span=0, dtype=np.float64)
        spr = oracle.aabb_pairs(sub.xyz, sub.offsets)
        t0 = time.perf_counter()
        ox, oo, of = oracle.discretize(sub.xyz, sub.offsets, spr)
        dt = time.perf_counter() - t0
        g = ctx.discretize(torch.from_numpy(sub.xyz).cuda(), torch.from_numpy(sub.offsets).cuda(),
                           torch.from_numpy(spr).cuda())
        leg["cpu_baseline"] = {
            "value": len(sub.xyz) / dt, "unit": "input spans/s", "cores": 1, "kind": "oracle",
            "sample": "first %d rows of the same workload (%d spans, %d pairs)" % (
                sub.n_loops, len(sub.xyz), len(spr)),
            "seconds": dt,
            "bitwise_equal_gpu": bool(np.array_equal(g[1].cpu().numpy(), oo)
                                      and np.array_equal(g[0].cpu().numpy().view(np.uint64),
                                                         ox.view(np.uint64))),
        }
    return leg


def run_serving(args):
    """--config serving: the serving leg as the headline line."""
    import torch
    torch.cuda.set_device(0)
    leg = serving_leg(args, args.requests, args.load, args.scenes, args.mode)
    line = {
        "metric": "segment-pair evals/s",
        "value": leg["value"],
        "unit": "segment-pairs/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": args.scenes,
        "ms_per_step": leg["latency"]["mean_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.mode == "plain" else ("f32 predicates+f64" if args.mode == "crossings"
                                                      else "f32+f64"),
        "data": "synthetic",
        "config": {"workload": "serving", "description": WORKLOADS["serving"],
                   "requests": args.requests, "load": args.load, "scenes": args.scenes,
                   "slots": 4, "seed": args.seed, "mode": args.mode},
    }
    line.update({k: v for k, v in leg.items() if k not in ("workload", "description", "value",
                                                             "unit", "mode")})
    print(json.dumps(line), flush=True)


def cpu_baseline(ls, pr, res, other, threads, cc=None):
    """Time the FP64 oracle on the host cores over a bounded sample of pairs
    (the whole pair list when it is small enough, timed over repeated passes
    for at least 10 s), and compare the GPU results on that sample with it."""
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = min(cores, 16) if threads <= 0 else threads
    sizes = ls.sizes.astype(np.int64)
    cost = sizes[pr[:, 0]] * sizes[pr[:, 1]]
    budget = 4.0e9  # terms: ~10-30 s on 16 host cores
    if cost.sum() <= budget:
        idx = np.arange(len(pr))
        sample = "all %d pairs" % len(pr)
    else:
        rng = np.random.default_rng(0)
        order = rng.permutation(len(pr))
        keep = order[np.cumsum(cost[order]) <= budget]
        idx = np.sort(keep)
        sample = "%d of %d pairs (seeded random, %.2e of %.2e terms)" % (
            len(idx), len(pr), cost[idx].sum(), cost.sum())
    t0 = time.perf_counter()
    oreal, olk = oracle.direct_sum(ls.xyz, ls.offsets, pr[idx], nthreads=cores)
    dt = time.perf_counter() - t0
    terms = int(cost[idx].sum())
    # a sample that finishes quickly is timed again, for at least 10 s in all
    passes = 1
    while dt < 10.0 and passes < 200 and len(idx):
        t1 = time.perf_counter()
        oracle.direct_sum(ls.xyz, ls.offsets, pr[idx], nthreads=cores)
        dt += time.perf_counter() - t1
        passes += 1
    timed = sample + (", timed over %d passes" % passes if passes > 1 else "")
    terms *= passes
    errs = {
        "err_vs_oracle": {
            "sample": sample,
            "mixed_max": float(np.max(np.abs(res["real"][idx] - oreal))) if len(idx) else 0.0,
            "mixed_p99": float(np.quantile(np.abs(res["real"][idx] - oreal), 0.99)) if len(idx) else 0.0,
            "int_mismatch": int(np.sum(res["lk"][idx] != olk)),
        }
    }
    if other is not None and len(idx):
        errs["err_vs_oracle"]["plain_max"] = float(np.max(np.abs(other["real"][idx] - oreal)))
        errs["err_vs_oracle"]["plain_int_mismatch"] = int(np.sum(other["lk"][idx] != olk))
    if cc is not None and len(idx):
        errs["err_vs_oracle"]["crossings_int_mismatch"] = int(np.sum(cc["lk"][idx] != olk))
    cpu = {"value": terms / dt, "unit": "segment-pairs/s", "cores": cores, "kind": "oracle",
           "sample": timed, "seconds": dt, "terms": terms, "threads": cores,
           "threads_rule": "the process's CPU affinity, at most 16 (the host share of one GPU)",
           "host": host_cpu(), "oracle_cflags": " ".join(oracle.CFLAGS)}
    return cpu, errs


def host_cpu():
    """Logical CPUs of the host, those this process may run on, and the model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.lower().startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = None
    return {"nproc": os.cpu_count(), "affinity": aff, "cpu_model": model}


if __name__ == "__main__":
    main()

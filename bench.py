"""Benchmark: threshold RHG generation throughput (edges/s) on one MI355X.

Workload (default): n = 10^7 points, alpha = 0.75 (degree exponent 2.5),
average degree 100 (R by getTargetRadius = 26.506...), SplitMix64 seed 1,
about 5.0e8 undirected edges written as int32 pairs (4 GB).  A step is one
whole generation through the C ABI: sample -> slab keys -> radix sort ->
table -> slab index -> window plan -> count -> scan -> emit into a
preallocated device buffer (rhg_count + rhg_emit).  The FP64 form gives
`value`; the FP32-filter + FP64-recheck form is timed the same way and
reported beside it (its edge list is checked byte-identical).

Also reported: per-phase device times (HIP events on the library stream),
the roofline of the dominant kernel, and the CPU oracle on a bounded sample
of the same workload (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edges/s at n=1e7, kbar=100 (FP64 vs FP32+recheck); p50/p99 request latency"
HBM_PEAK_GBS = 8000.0


def kernel_bytes(n, windows, units, m):
    """Algorithmic HBM bytes per launch of the two query kernels:
    count reads the 5 FP64 table columns once per point (40 B), each window
    record (8 B) and writes one count per unit (4 B); emit reads the same plus
    the original index (4 B per point) and writes one int32 pair per edge (8 B)."""
    count = 40 * n + 8 * windows + 4 * units
    emit = 44 * n + 8 * windows + 8 * m
    return count, emit


def run_gpu(args):
    import torch
    from paper_1606_09481_amd import rhg

    rhg.load()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = rhg.rhg_ctx_create(0, stream)
    res = {}
    out = None
    ref_edges = None
    for prec, name in ((rhg.RHG_FP64, "fp64"), (rhg.RHG_FP32_RECHECK, "fp32_recheck")):
        p = rhg.params(args.n, args.alpha, kbar=args.kbar, seed=args.seed, precision=prec)
        times, stats = [], []
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan, m = rhg.rhg_count(ctx, p)
            if out is None or out.numel() < 2 * m:
                del out
                out = None
                torch.cuda.synchronize()
                out = torch.empty(2 * m + 1024, dtype=torch.int32, device="cuda")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rhg.rhg_graph_free(plan)
                plan, m = rhg.rhg_count(ctx, p)
            rhg.rhg_emit(ctx, plan, out, out.numel() // 2)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = rhg.rhg_graph_stats(plan)
            R = rhg.rhg_graph_radius(plan)
            rhg.rhg_graph_free(plan)
            if it >= args.warmup:
                times.append(t1 - t0)
                stats.append(st)
            print("[bench] %s step %d: %.3f ms, m=%d" % (name, it, 1e3 * (t1 - t0), m), file=sys.stderr, flush=True)
        if name == "fp64":
            ref_edges = out[: 2 * m].clone()
        else:
            same = bool(torch.equal(out[: 2 * m], ref_edges))
            res["fp32_identical_to_fp64"] = same
        avg = lambda k: sum(s["ms"][k] for s in stats) / len(stats)
        T = sum(times) / len(times)
        res[name] = {
            "m": m, "R": R, "s_per_step": T, "edges_per_s": m / T,
            "phases_ms": {"keys": avg(0), "sort": avg(1), "table_index": avg(2), "plan_units": avg(3),
                          "count": avg(4), "edge_scan": avg(5), "emit": avg(6), "device_total": avg(7)},
            "candidates": stats[0]["candidates"], "windows": stats[0]["windows"],
            "rechecks": stats[0]["rechecks"],
            "units": None,
        }
    rhg.rhg_ctx_destroy(ctx)
    del out, ref_edges
    return res


def cpu_baseline(args, m_full):
    """The oracle as it stands on the host cores: sample + table + slab sort of
    all n points timed in full; the band sweep on the first `frac` of the
    queries (i.i.d. points: a uniform sample), scaled by 1/frac."""
    import oracle
    frac = args.cpu_frac
    threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    R = oracle.target_radius(args.n, args.alpha, args.kbar)
    th, r = oracle.sample(args.n, args.alpha, R, args.seed)
    tab = oracle.table(th, r)
    t1 = time.perf_counter()
    oracle.band_sweep(th, r, tab, R, math.cosh(R), threads=threads, q0=0, q1=0)   # slab sort alone
    t2 = time.perf_counter()
    q1 = int(args.n * frac)
    e = oracle.band_sweep(th, r, tab, R, math.cosh(R), threads=threads, q0=0, q1=q1)
    t3 = time.perf_counter()
    setup = (t1 - t0) + (t2 - t1)
    sweep = max((t3 - t2) - (t2 - t1), 1e-9)
    T_full = setup + sweep / frac
    m_est = len(e) / frac
    return {"value": m_est / T_full, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": "n=%d alpha=%g kbar=%g seed=%d: sampling, table and slab sort of all points timed in full "
                      "(%.1f s); band sweep over queries [0, %d) (%.0f%%, %d edges, %.1f s) scaled by 1/%.2f; "
                      "projected %.1f s for ~%.3g edges" % (args.n, args.alpha, args.kbar, args.seed, setup, q1,
                                                            100 * frac, len(e), t3 - t2, frac, T_full, m_est)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--alpha", type=float, default=0.75)
    ap.add_argument("--kbar", type=float, default=100.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-frac", type=float, default=0.1)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this generator runs on one GPU; multi-GPU sharding is not built (see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    res = run_gpu(args)
    f64, f32 = res["fp64"], res["fp32_recheck"]
    n = args.n
    cnt_b, emit_b = kernel_bytes(n, f64["windows"], 0, f64["m"])
    ph = f64["phases_ms"]
    if ph["emit"] >= ph["count"]:
        kname, kbytes, kms = "k_query<emit,fp64>", emit_b, ph["emit"]
    else:
        kname, kbytes, kms = "k_query<count,fp64>", cnt_b, ph["count"]
    achieved = kbytes / (kms * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": kbytes, "avg_ms": kms}
    line = {
        "metric": METRIC, "value": f64["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * f64["s_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "threshold RHG generation n=%d alpha=%g kbar=%g seed=%d (R=%.9f, %d edges)"
                               % (n, args.alpha, args.kbar, args.seed, f64["R"], f64["m"]),
                   "n": n, "alpha": args.alpha, "kbar": args.kbar, "R": f64["R"], "edges": f64["m"],
                   "candidates": f64["candidates"], "windows": f64["windows"]},
        "phases_ms": ph,
        "fp32_recheck": {"value": f32["edges_per_s"], "ms_per_step": 1e3 * f32["s_per_step"],
                         "rechecks": f32["rechecks"], "recheck_fraction": f32["rechecks"] / max(1, f32["candidates"]),
                         "identical_to_fp64": res.get("fp32_identical_to_fp64"), "phases_ms": f32["phases_ms"]},
        "roofline": roof,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args, f64["m"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

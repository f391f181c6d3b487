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
the roofline of the dominant kernel (and the other query kernel, and the
whole step), the CPU oracle on the same workload (cpu_baseline: the whole
generation on the host cores, median of 3), the other fixed workloads
(configs: n = 10^6 and the exponent sweep at n = 4 10^6, both precision
forms, recheck fractions, HBM fractions), the FP32 ablation (fp32_ablation:
the filter used against Eq. 3 as printed in FP32), the general model at
T > 0 (soft), the request server on a stream of 2000 mixed requests
(serving): closed-loop saturation throughput X, then Poisson arrivals at
0.7 X and at fixed rates with p50/p99 latency and aggregate edges/s; one
GPU's share of an 8-GPU run (share: whole table, 1/8 of the queries); the
dynamic model's movement step with the update and the regeneration of the
moved graph (dynamic); and the CSR adjacency (csr).
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


def kernel_bytes(n, m):
    """Algorithmic HBM bytes per launch of the two query kernels, as the
    method needs them (per point and per edge, independent of the plan):
    count reads the sorted FP64 table once (6 x 8 B per point: angle, exp(r),
    exp(-r), sinh r, sin and cos of the half angle) and writes a count per
    point (4 B); emit reads the table once more, the offsets (8 B per point)
    and writes one int32 pair per edge (8 B)."""
    count = 52 * n
    emit = 56 * n + 8 * m
    return count, emit


def step_bytes(n, m):
    """Algorithmic HBM bytes of one whole generation: read the coordinates
    (16 B per point), write the sorted table (48 B) and read it in count and
    emit (2 x 48 B), counts and offsets (12 B), and the edges (8 B each):
    172 B per point + 8 B per edge."""
    return 172 * n + 8 * m


def run_gpu(args, n=None, alpha=None, kbar=None, steps=None, warmup=None, tag=""):
    """Times `steps` whole generations (after `warmup`) in each precision form
    through rhg_count + rhg_emit into one preallocated device buffer."""
    import torch
    from paper_1606_09481_amd import rhg

    n = args.n if n is None else n
    alpha = args.alpha if alpha is None else alpha
    kbar = args.kbar if kbar is None else kbar
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    rhg.load()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = rhg.rhg_ctx_create(0, stream)
    res = {}
    out = None
    ref_edges = None
    for prec, name in ((rhg.RHG_FP64, "fp64"), (rhg.RHG_FP32_RECHECK, "fp32_recheck")):
        p = rhg.params(n, alpha, kbar=kbar, seed=args.seed, precision=prec)
        times, stats = [], []
        for it in range(warmup + steps):
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
            if it >= warmup:
                times.append(t1 - t0)
                stats.append(st)
            print("[bench] %s%s step %d: %.3f ms, m=%d" % (tag, name, it, 1e3 * (t1 - t0), m), file=sys.stderr,
                  flush=True)
        if name == "fp64":
            ref_edges = out[: 2 * m].clone()
        else:
            same = bool(torch.equal(out[: 2 * m], ref_edges))
            res["fp32_identical_to_fp64"] = same
        avg = lambda k: sum(s["ms"][k] for s in stats) / len(stats)
        T = sum(times) / len(times)
        res[name] = {
            "m": m, "R": R, "s_per_step": T, "edges_per_s": m / T,
            "count_kernel_ms": sum(s["count_kernel_ms"] for s in stats) / len(stats),
            "phases_ms": {"keys": avg(0), "sort": avg(1), "table_index": avg(2), "plan_units": avg(3),
                          "count": avg(4), "edge_scan": avg(5), "emit": avg(6), "device_total": avg(7)},
            "candidates": stats[0]["candidates"], "windows": stats[0]["windows"],
            "rechecks": stats[0]["rechecks"],
            "units": None,
        }
    rhg.rhg_ctx_destroy(ctx)
    del out, ref_edges
    torch.cuda.empty_cache()
    return res


def run_shares(args):
    """One GPU's share of an S-GPU run of the same workload: the whole table is
    sampled, sorted and planned, count and emit cover the batches of share k
    (cut on the plan's candidate prefix).  Host-timed like the main step."""
    import torch
    from paper_1606_09481_amd import rhg

    S = args.shares
    rhg.load()
    torch.cuda.set_device(0)
    ctx = rhg.rhg_ctx_create(0, torch.cuda.current_stream())
    rhg.rhg_ctx_set_option(ctx, rhg.RHG_OPT_SHARD_COUNT, S)
    p = rhg.params(args.n, args.alpha, kbar=args.kbar, seed=args.seed)
    out, per = None, []
    try:
        for k in range(S):
            rhg.rhg_ctx_set_option(ctx, rhg.RHG_OPT_SHARD_INDEX, k)
            times = []
            for it in range(1 + 2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan, m = rhg.rhg_count(ctx, p)
                if out is None or out.numel() < 2 * m:
                    rhg.rhg_graph_free(plan)
                    out = None
                    torch.cuda.synchronize()
                    out = torch.empty(2 * m + 1024, dtype=torch.int32, device="cuda")
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    plan, m = rhg.rhg_count(ctx, p)
                rhg.rhg_emit(ctx, plan, out, out.numel() // 2)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st = rhg.rhg_graph_stats(plan)
                rhg.rhg_graph_free(plan)
                if it >= 1:
                    times.append(t1 - t0)
            per.append({"edges": m, "candidates": st["candidates"], "ms": 1e3 * sum(times) / len(times),
                        "count_ms": st["ms"][4], "emit_ms": st["ms"][6]})
            print("[bench] share %d/%d: %.3f ms, m=%d" % (k, S, per[-1]["ms"], m), file=sys.stderr, flush=True)
    finally:
        rhg.rhg_ctx_destroy(ctx)
        del out
        torch.cuda.empty_cache()
    return {"count": S, "what": "whole table sampled, sorted and planned; count and emit for 1/%d of the "
                                "queries (by candidates)" % S,
            "max_ms": max(x["ms"] for x in per), "mean_ms": sum(x["ms"] for x in per) / S, "shares": per}


def run_csr(args):
    """Symmetric CSR adjacency (rhg_csr_from_pairs) of the benchmark graph: the
    FP64 edge list emitted into a device tensor, then rows and columns built
    on the device (host-timed, synchronous call; 1 warm-up + 3 timed)."""
    import torch
    from paper_1606_09481_amd import rhg

    rhg.load()
    torch.cuda.set_device(0)
    ctx = rhg.rhg_ctx_create(0, torch.cuda.current_stream())
    try:
        p = rhg.params(args.n, args.alpha, kbar=args.kbar, seed=args.seed, precision=rhg.RHG_FP64)
        plan, m = rhg.rhg_count(ctx, p)
        pairs = torch.empty(2 * m, dtype=torch.int32, device="cuda")
        rhg.rhg_emit(ctx, plan, pairs, m)
        rhg.rhg_graph_free(plan)
        row_ptr = torch.empty(args.n + 1, dtype=torch.int64, device="cuda")
        col = torch.empty(2 * m, dtype=torch.int32, device="cuda")
        ts = []
        for it in range(1 + 3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rhg.rhg_csr_from_pairs(ctx, args.n, pairs, m, row_ptr, col)
            t1 = time.perf_counter()
            if it >= 1:
                ts.append(t1 - t0)
        t = sum(ts) / len(ts)
        deg = row_ptr[1:] - row_ptr[:-1]
        res = {"ms": 1e3 * t, "edges": m, "entries": 2 * m, "entries_per_s": 2 * m / t,
               "max_degree": int(deg.max().item()), "isolated": int((deg == 0).sum().item()),
               "what": "rhg_csr_from_pairs: 2 directed entries per edge, stable radix sort by row, row pointers"}
        del pairs, row_ptr, col, deg
    finally:
        rhg.rhg_ctx_destroy(ctx)
        torch.cuda.empty_cache()
    return res


def run_dynamic(args):
    """Dynamic model (Sec. III-C) at the benchmark size: one movement step of
    all nodes and of 12% of them (tau_phi in (-1, 1), tau_r in (-10, 1), the
    paper's ranges), timed with HIP events on the context stream; then one
    more 12% move, whose graph is both updated from the graph before it and
    regenerated from the device arrays."""
    import torch
    from paper_1606_09481_amd import rhg

    rhg.load()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = rhg.rhg_ctx_create(0, stream)
    n, alpha = args.n, args.alpha
    R = rhg.rhg_target_radius(n, alpha, args.kbar)
    g = torch.Generator(device="cuda").manual_seed(args.seed)
    u = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
    th = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * (2 * math.pi)
    r = (2.0 * torch.asinh(torch.sqrt(u) * math.sinh(alpha * R / 2.0)) / alpha).clamp_(max=R)  # Eq. 1
    res = {"n": n, "R": R, "bytes_per_node": 48}
    try:
        for frac in (1.0, 0.12):
            sel = torch.rand(n, device="cuda", generator=g) < frac
            tp = torch.where(sel, torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 2 - 1, 0.0)
            tr = torch.where(sel, torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 11 - 10, 0.0)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            times = []
            for it in range(2 + 10):
                ev[0].record(stream)
                rhg.rhg_move(ctx, th, r, tp, tr, alpha, R)
                ev[1].record(stream)
                torch.cuda.synchronize()
                if it >= 2:
                    times.append(ev[0].elapsed_time(ev[1]))
            t = sum(times) / len(times)
            gbs = 48.0 * n / (t * 1e-3) / 1e9  # read theta, r, tau_phi, tau_r; write theta, r
            res["move_all" if frac == 1.0 else "move_12pct"] = {"ms": t, "GB_s": gbs, "frac_of_hbm_peak": gbs / 8000.0}
        # the graph before one more 12% move, then the graph after it: updated
        # (rhg_update_after_move) and regenerated (rhg_generate_from_coords)
        g0 = rhg.rhg_generate_from_coords(ctx, th, r, R)
        m0 = rhg.rhg_graph_num_edges(g0)
        old = rhg.rhg_graph_edges_device(g0)
        sel = torch.rand(n, device="cuda", generator=g) < 0.12
        tp = torch.where(sel, torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 2 - 1, 0.0)
        tr = torch.where(sel, torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 11 - 10, 0.0)
        moved = sel.to(torch.uint8)
        rhg.rhg_move(ctx, th, r, tp, tr, alpha, R)
        upd, gen = [], []
        for it in range(1 + 3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gu = rhg.rhg_update_after_move(ctx, th, r, R, moved, old, m0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            mu = rhg.rhg_graph_num_edges(gu)
            st_u = rhg.rhg_graph_stats(gu)
            rhg.rhg_graph_free(gu)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            gr = rhg.rhg_generate_from_coords(ctx, th, r, R)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            m = rhg.rhg_graph_num_edges(gr)
            rhg.rhg_graph_free(gr)
            if it >= 1:
                upd.append(t1 - t0)
                gen.append(t3 - t2)
        rhg.rhg_graph_free(g0)
        if mu != m:
            raise RuntimeError("update after a move gave %d edges, regeneration %d" % (mu, m))
        res["regenerate"] = {"ms": 1e3 * sum(gen) / len(gen), "edges": m,
                             "what": "rhg_generate_from_coords on the moved device arrays (library-owned output)"}
        res["update_12pct"] = {"ms": 1e3 * sum(upd) / len(upd), "edges": mu, "edges_before": m0,
                               "moved": int(sel.sum().item()), "device_phases_ms": st_u.get("ms"),
                               "speedup_vs_regenerate": sum(gen) / sum(upd),
                               "what": "rhg_update_after_move from the graph before a move of 12% of the nodes "
                                       "(library-owned output; same edge count as the regeneration)"}
    finally:
        rhg.rhg_ctx_destroy(ctx)
        del th, r, u
        torch.cuda.empty_cache()
    return res


def summarize(res, n):
    """Edges/s of both precision forms, the recheck fraction and the HBM
    fractions (algorithmic bytes over time) of one timed configuration."""
    f64, f32 = res["fp64"], res["fp32_recheck"]
    m = f64["m"]
    cb, eb = kernel_bytes(n, m)
    sb = step_bytes(n, m)
    frac = lambda b, ms: b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    return {
        "edges": m, "R": f64["R"], "candidates": f64["candidates"], "windows": f64["windows"],
        "fp64": {"edges_per_s": f64["edges_per_s"], "ms_per_step": 1e3 * f64["s_per_step"],
                 "count_kernel_ms": f64["count_kernel_ms"], "emit_ms": f64["phases_ms"]["emit"],
                 "device_ms": f64["phases_ms"]["device_total"]},
        "fp32_recheck": {"edges_per_s": f32["edges_per_s"], "ms_per_step": 1e3 * f32["s_per_step"],
                         "count_kernel_ms": f32["count_kernel_ms"], "rechecks": f32["rechecks"],
                         "recheck_fraction": f32["rechecks"] / max(1, f32["candidates"]),
                         "identical_to_fp64": res.get("fp32_identical_to_fp64")},
        "hbm_frac": {"step": frac(sb, 1e3 * f64["s_per_step"]), "count": frac(cb, f64["count_kernel_ms"]),
                     "emit": frac(eb, f64["phases_ms"]["emit"]), "step_bytes": sb,
                     "what": "algorithmic bytes (172 B/point + 8 B/edge per step; count 52 B/point; emit "
                             "56 B/point + 8 B/edge) over the FP64 host step time and the kernels' HIP-event "
                             "times, against 8 TB/s"},
    }


CONFIGS = [(1_000_000, 1.0, 20.0), (4_000_000, 0.55, 64.0), (4_000_000, 1.0, 64.0), (4_000_000, 1.5, 64.0)]


def run_configs(args):
    """The other fixed workloads: n = 10^6, alpha = 1, kbar = 20 and the
    exponent sweep n = 4 10^6, kbar = 64, alpha in {0.55, 1, 1.5}, both
    precision forms (2 warm-up + 5 timed steps each)."""
    out = {}
    for (n, alpha, kbar) in CONFIGS:
        res = run_gpu(args, n=n, alpha=alpha, kbar=kbar, steps=5, warmup=2, tag="n=%d a=%g " % (n, alpha))
        out["n=%d alpha=%g kbar=%g" % (n, alpha, kbar)] = summarize(res, n)
    return out


def run_ablation(args):
    """The FP32 forms side by side on every candidate of one generation:
    the cancellation-free filter actually used (its margin mu = 2^-20 leaves
    `recheck_fraction` undecided) against Eq. 3 as printed in FP32
    (undecided under its sound margin 8 u32 (A + S), and the error rate of
    its plain FP32 decision against the FP64 test)."""
    from paper_1606_09481_amd import rhg
    import torch
    rhg.load()
    ctx = rhg.rhg_ctx_create(0, torch.cuda.current_stream())
    rhg.rhg_ctx_set_option(ctx, rhg.RHG_OPT_LITERAL_ABLATION, 1)
    out = {}
    try:
        for (n, alpha, kbar) in [(args.n, args.alpha, args.kbar)] + CONFIGS:
            plan, m = rhg.rhg_count(ctx, rhg.params(n, alpha, kbar=kbar, seed=args.seed,
                                                    precision=rhg.RHG_FP32_RECHECK))
            st = rhg.rhg_graph_stats(plan)
            rhg.rhg_graph_free(plan)
            c = max(1, st["candidates"])
            out["n=%d alpha=%g kbar=%g" % (n, alpha, kbar)] = {
                "candidates": st["candidates"], "edges": m,
                "filter_recheck_fraction": st["rechecks"] / c, "filter_disagreements": st["disagreements"],
                "literal_undecided_fraction": st["literal_undecided"] / c,
                "literal_raw_error_rate": st["literal_wrong"] / c}
            print("[bench] ablation n=%d alpha=%g: filter rechecks %.2e, literal undecided %.3f, literal wrong %.2e"
                  % (n, alpha, st["rechecks"] / c, st["literal_undecided"] / c, st["literal_wrong"] / c),
                  file=sys.stderr, flush=True)
    finally:
        rhg.rhg_ctx_destroy(ctx)
    return out


SOFT_CONFIGS = [(1_000_000, 1.0, 20.0, 0.1), (10_000_000, 0.75, 100.0, 0.05)]


def run_soft(args):
    """The general model at temperature T > 0 (Eq. 2): rhg_count_soft +
    rhg_emit into a preallocated buffer, 1 warm-up + 3 timed steps."""
    import torch
    from paper_1606_09481_amd import rhg
    rhg.load()
    ctx = rhg.rhg_ctx_create(0, torch.cuda.current_stream())
    res = {}
    out = None
    try:
        for (n, alpha, kbar, T) in SOFT_CONFIGS:
            p = rhg.params(n, alpha, kbar=kbar, seed=args.seed)
            ts = []
            for it in range(1 + 3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan, m = rhg.rhg_count_soft(ctx, p, T)
                if out is None or out.numel() < 2 * m:
                    rhg.rhg_graph_free(plan)
                    out = None
                    torch.cuda.synchronize()
                    out = torch.empty(2 * m + 1024, dtype=torch.int32, device="cuda")
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    plan, m = rhg.rhg_count_soft(ctx, p, T)
                rhg.rhg_emit(ctx, plan, out, out.numel() // 2)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st = rhg.rhg_graph_stats(plan)
                R = rhg.rhg_graph_radius(plan)
                rhg.rhg_graph_free(plan)
                if it >= 1:
                    ts.append(t1 - t0)
            t = sum(ts) / len(ts)
            res["n=%d alpha=%g kbar=%g T=%g" % (n, alpha, kbar, T)] = {
                "edges_per_s": m / t, "ms_per_step": 1e3 * t, "edges": m, "avg_degree": 2.0 * m / n, "R": R,
                "candidates": st["candidates"], "candidates_per_edge": st["candidates"] / max(1, m),
                "count_kernel_ms": st["count_kernel_ms"], "emit_ms": st["ms"][6]}
            print("[bench] soft n=%d T=%g: %.3f ms, m=%d, %.1f candidates/edge" % (
                n, T, 1e3 * t, m, st["candidates"] / max(1, m)), file=sys.stderr, flush=True)
    finally:
        rhg.rhg_ctx_destroy(ctx)
        del out
        torch.cuda.empty_cache()
    return res


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "query_traffic_n1e7_a075_k100.md")
KERNEL_SOURCES = ["query_dev.h", "query.hip", "rhg_device.h", "rhg_kernels.h"]


ISSUE_FILE = os.path.join(ROOT, "profiles", "query_issue_n1e7_a075_k100.md")
# SIMD cycles per second: 256 CUs x 4 SIMDs x 2.4 GHz.  A wavefront VALU
# instruction takes 2 of them for 32-bit operations (the FP32 vector peak,
# 157.3 TFLOP/s = 256 x 128 FMA lanes x 2 x 2.4 GHz) and 4 for FP64
# arithmetic (78.6 TFLOP/s).
VALU_CYCLE_PEAK = 256 * 4 * 2.4e9


def measured_traffic(key, path=TRAFFIC_FILE, tag="traffic"):
    """HBM bytes per launch of kernel `key` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the kernel sources
    no longer hash to the ones the counters were taken with.  With
    path=ISSUE_FILE, tag="valu": its VALU instructions per launch."""
    import hashlib
    try:
        lines = open(path).read().split("\n")
    except OSError:
        return None, None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1606_09481_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    want = [l.split()[1] for l in lines if l.strip().startswith("sources_sha256")]
    if not want or want[0] != h.hexdigest():
        return None, "counters taken with other kernel sources"
    for l in lines:
        t = l.split()
        if len(t) == 3 and t[0] == tag and t[1] == key:
            return int(t[2]), os.path.relpath(path, ROOT)
    return None, None


def copy_calibration(mib):
    """Three device-to-device copies of mib MiB: each reads and writes exactly
    mib MiB, the reference for FETCH_SIZE / WRITE_SIZE per dispatch."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("[bench] copy calibration: 3 x %d MiB device copies" % mib, file=sys.stderr, flush=True)


def serving_requests(rhg, count, seed):
    """The serving mix: n log-uniform in [1e3, 2e6], alpha uniform in
    [0.55, 1.5], kbar uniform integer in 6..64 (combinations whose average
    degree the model cannot reach are drawn again), request i seeded base+i;
    every third request in the FP32-filter form, the others FP64."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e6)))))
        alpha = float(rng.uniform(0.55, 1.5))
        kbar = float(rng.integers(6, 65))
        try:
            rhg.rhg_target_radius(n, alpha, kbar)
        except rhg.RhgError:
            continue
        prec = rhg.RHG_FP32_RECHECK if len(out) % 3 == 2 else rhg.RHG_FP64
        out.append(rhg.params(n, alpha, kbar=kbar, seed=1000 + len(out), precision=prec))
    return out


def poisson_arrivals(count, rate, seed):
    """Arrival times (s) of a Poisson process of the given rate, reproducible from its seed."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def _serve(rhg, srv, reqs, arrivals):
    """Submits reqs[i] at arrivals[i] seconds (None: all at once) from a
    submitter thread; collects in order.  Returns (wall s, latencies ms, edges)."""
    import queue
    import threading
    q = queue.Queue()
    t_start = time.perf_counter()

    def submitter():
        for i, p in enumerate(reqs):
            if arrivals is not None:
                d = t_start + arrivals[i] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
            q.put(rhg.rhg_server_submit(srv, p))

    th = threading.Thread(target=submitter)
    th.start()
    lat, edges = [], 0
    for _ in reqs:
        g, ms = rhg.rhg_server_wait(srv, q.get())
        edges += rhg.rhg_graph_num_edges(g)
        rhg.rhg_graph_free(g)
        lat.append(ms)
    th.join()
    return time.perf_counter() - t_start, lat, edges


def run_serving(args):
    import numpy as np
    from paper_1606_09481_amd import rhg
    rhg.load()
    reqs = serving_requests(rhg, args.serve_requests, args.seed)
    small = np.array([p.n <= 16384 for p in reqs])
    srv = rhg.rhg_server_create(0, args.serve_budget_gb << 30)
    try:
        _serve(rhg, srv, reqs[:100], None)  # warm-up: lane buffers, code objects
        T_sat, lat_sat, edges = _serve(rhg, srv, reqs, None)
        X = len(reqs) / T_sat
        lam = 0.7 * X
        arrivals = poisson_arrivals(len(reqs), lam, args.seed + 7)
        T, lat, edges2 = _serve(rhg, srv, reqs, arrivals)
        # the same stream at a fixed arrival rate, comparable across runs
        fixed = {}
        for rate in args.serve_rates:
            Tf, latf, edgesf = _serve(rhg, srv, reqs, poisson_arrivals(len(reqs), rate, args.seed + 7))
            latf = np.array(latf)
            fixed["%g" % rate] = {"p50": float(np.percentile(latf, 50)), "p99": float(np.percentile(latf, 99)),
                                  "mean": float(latf.mean()), "edges_per_s": edgesf / Tf,
                                  "achieved_req_per_s": len(reqs) / Tf}
            print("[bench] serving at %.0f req/s: p50 %.3f ms p99 %.3f ms" % (rate, fixed["%g" % rate]["p50"],
                  fixed["%g" % rate]["p99"]), file=sys.stderr, flush=True)
        cnt = rhg.rhg_server_counters(srv)
    finally:
        rhg.rhg_server_destroy(srv)
    lat = np.array(lat)
    pct = lambda a, q: float(np.percentile(a, q)) if len(a) else None
    print("[bench] serving: saturation %.1f req/s (%.3g edges/s), open loop at %.1f req/s: p50 %.3f ms p99 %.3f ms"
          % (X, edges / T_sat, lam, pct(lat, 50), pct(lat, 99)), file=sys.stderr, flush=True)
    return {
        "requests": len(reqs), "edges": int(edges), "budget_bytes": args.serve_budget_gb << 30,
        "mix": "n log-uniform [1e3, 2e6], alpha U[0.55, 1.5], kbar U{6..64}, request i seed 1000+i, "
               "every third request FP32 filter + FP64 recheck, the others FP64",
        "saturation_req_per_s": X, "saturation_edges_per_s": edges / T_sat,
        "arrival_rate_req_per_s": lam, "arrivals": "Poisson, seed %d" % (args.seed + 7),
        "edges_per_s": edges2 / T, "wall_s": T,
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "mean": float(lat.mean()), "max": float(lat.max()),
                       "small_p50": pct(lat[small], 50), "small_p99": pct(lat[small], 99),
                       "large_p50": pct(lat[~small], 50), "large_p99": pct(lat[~small], 99)},
        "latency_definition": "submit (at arrival) to results host-visible after the device finished",
        "fixed_rate": fixed, "fixed_rate_arrivals": "Poisson at the stated rate (req/s), seed %d" % (args.seed + 7),
        "small_fraction": float(small.mean()), "counters": cnt,
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(args, m_full):
    """The oracle as it stands on the host cores: sampling, table, slab sort
    and the band sweep over every query of the benchmark workload, timed in
    full `cpu_runs` times on all the cores the job may use (median); and on
    one thread, the same phases with the sweep over 1% of the queries (i.i.d.
    points: a uniform sample), scaled by 100 (a labelled projection)."""
    import oracle
    threads = oracle.default_threads()
    R = oracle.target_radius(args.n, args.alpha, args.kbar)
    runs = []
    m = None
    for k in range(max(1, args.cpu_runs)):
        t0 = time.perf_counter()
        th, r = oracle.sample(args.n, args.alpha, R, args.seed, threads=threads)
        tab = oracle.table(th, r, threads=threads)
        e = oracle.band_sweep(th, r, tab, R, math.cosh(R), threads=threads)
        t1 = time.perf_counter()
        m = len(e)
        runs.append(t1 - t0)
        del th, r, tab, e
        print("[bench] cpu oracle run %d: %.2f s, m=%d" % (k, t1 - t0, m), file=sys.stderr, flush=True)
    T_med = sorted(runs)[len(runs) // 2]
    # one thread: whole setup, sweep over 1% of the queries
    f1 = 0.01
    q1s = int(args.n * f1)
    t3 = time.perf_counter()
    th1, r1 = oracle.sample(args.n, args.alpha, R, args.seed, threads=1)
    tab1 = oracle.table(th1, r1, threads=1)
    t4 = time.perf_counter()
    oracle.band_sweep(th1, r1, tab1, R, math.cosh(R), threads=1, q0=0, q1=0)
    t5 = time.perf_counter()
    e1 = oracle.band_sweep(th1, r1, tab1, R, math.cosh(R), threads=1, q0=0, q1=q1s)
    t6 = time.perf_counter()
    sweep1 = max((t6 - t5) - (t5 - t4), 1e-9)
    T1 = (t4 - t3) + (t5 - t4) + sweep1 / f1
    m1 = len(e1) / f1
    return {"value": m / T_med, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": "n=%d alpha=%g kbar=%g seed=%d, the whole generation: sampling, table, slab sort and the "
                      "band sweep over every query (%d edges; the GPU's m = %d), median of %d runs on %d threads "
                      "(%s s)" % (args.n, args.alpha, args.kbar, args.seed, m, m_full, len(runs), threads,
                                  ", ".join("%.2f" % x for x in runs)),
            "single_thread": {"value": m1 / T1, "unit": "edges/s", "cores": 1, "kind": "oracle, projected",
                              "sample": "sampling, table and slab sort of all points on one thread (%.1f s); "
                                        "band sweep over queries [0, %d) (1%%, %d edges, %.1f s) scaled by 100; "
                                        "projected %.1f s for the whole generation" % (t5 - t3, q1s, len(e1),
                                                                                      t6 - t5, T1)}}


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
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-only", action="store_true", help="only the serving stream (prints its JSON)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the steps, copy a MIB-MiB device buffer 3 times (the known-size kernel that "
                         "scales HBM byte counters under rocprofv3 --pmc)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-budget-gb", type=int, default=32)
    ap.add_argument("--serve-rates", type=float, nargs="*", default=[6000.0, 8000.0],
                    help="fixed Poisson arrival rates (req/s) at which to also report latency")
    ap.add_argument("--no-configs", action="store_true", help="skip the n = 1e6 and n = 4e6 workloads")
    ap.add_argument("--no-ablation", action="store_true", help="skip the literal-Eq. 3 FP32 ablation")
    ap.add_argument("--no-soft", action="store_true", help="skip the T > 0 workloads")
    ap.add_argument("--cpu-runs", type=int, default=3, help="full oracle runs for cpu_baseline (median)")
    ap.add_argument("--no-dynamic", action="store_true", help="skip the dynamic-model timing")
    ap.add_argument("--no-csr", action="store_true", help="skip the CSR adjacency timing")
    ap.add_argument("--shares", type=int, default=8,
                    help="also time each of this many one-GPU query shares (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; the 'share' object of its JSON line times one GPU's share "
              "of a multi-GPU run (no collectives are built)", file=sys.stderr)
        sys.exit(2)

    if args.serve_only:
        print(json.dumps({"serving": run_serving(args)}), flush=True)
        return
    # the request stream runs first: after the 4 GB edge buffers of the main
    # step have come and gone, this process serves about 15% fewer requests
    serving = run_serving(args) if not args.no_serve else None
    res = run_gpu(args)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    f64, f32 = res["fp64"], res["fp32_recheck"]
    n = args.n
    cnt_b, emit_b = kernel_bytes(n, f64["m"])
    ph = f64["phases_ms"]
    bench_cfg = (n, args.alpha, args.kbar, args.seed) == (10_000_000, 0.75, 100.0, 1)

    def roofline(kname, kkey, kbytes, kms):
        achieved = kbytes / (kms * 1e-3) / 1e9
        traffic, traffic_src = measured_traffic(kkey) if bench_cfg else (None, None)
        return {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes": kbytes, "avg_ms": kms,
                "traffic_source": traffic_src,
                # the measured bytes over the same time: the second fraction the workload's roofline asks for
                "traffic_frac": (traffic / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None}

    # the dominant kernel is the longer of the two query kernels of the timed FP64 step
    r_emit = roofline("k_emit<false,false>", "k_emit", emit_b, ph["emit"])
    r_count = roofline("k_count<0,false,false>", "k_count", cnt_b, f64["count_kernel_ms"])
    roof, other = (r_emit, r_count) if ph["emit"] >= f64["count_kernel_ms"] else (r_count, r_emit)

    def issue(kname, kkey, kms):
        # the same kernel against the chip's VALU cycles: its wavefront VALU
        # instructions per launch (committed SQ_INSTS_VALU and FP64 counts) at
        # 2 SIMD cycles each, 4 for FP64 arithmetic, over its time
        n_valu, src = measured_traffic(kkey, ISSUE_FILE, "valu") if bench_cfg else (None, None)
        n_f64, _ = measured_traffic(kkey, ISSUE_FILE, "valu_f64") if bench_cfg else (None, None)
        if n_valu is None or n_f64 is None:
            return {"bound": "alu", "kernel": kname, "achieved": None, "source": src}
        cycles = 2 * (n_valu - n_f64) + 4 * n_f64
        achieved = cycles / (kms * 1e-3)
        return {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": VALU_CYCLE_PEAK,
                "unit": "SIMD VALU cycles/s", "frac": achieved / VALU_CYCLE_PEAK,
                "valu_instructions": n_valu, "valu_f64_instructions": n_f64, "valu_cycles": cycles,
                "avg_ms": kms, "source": src}

    issues = [issue("k_count<0,false,false>", "k_count", f64["count_kernel_ms"]),
              issue("k_emit<false,false>", "k_emit", ph["emit"]),
              issue("k_count<1,false,false>", "k_count_fp32", f32["count_kernel_ms"])]
    if roof is r_count and issues[0].get("achieved") is not None:
        # the count kernel is bound on chip (it reads 52 B per point from HBM): when it is the
        # longer kernel, its binding roofline is the VALU cycles, with its HBM view beside it
        roof = dict(issues[0], traffic=r_count["traffic"], hbm=r_count)
    roof = dict(roof, other=other, issue=issues)
    line = {
        "metric": METRIC, "value": f64["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * f64["s_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "threshold RHG generation n=%d alpha=%g kbar=%g seed=%d (R=%.9f, %d edges)"
                               % (n, args.alpha, args.kbar, args.seed, f64["R"], f64["m"]),
                   "n": n, "alpha": args.alpha, "kbar": args.kbar, "R": f64["R"], "edges": f64["m"],
                   "candidates": f64["candidates"], "windows": f64["windows"],
                   "candidates_per_edge": f64["candidates"] / max(1, f64["m"])},
        "phases_ms": ph,
        # edges over the device time of slabs through emit only (Alg. 1 on a sampled, tabulated point set:
        # the sample + key phase and the table phase excluded); `value` above is the whole generation
        "edges_per_s_slabs_to_emit": f64["m"] / ((ph["device_total"] - ph["keys"] - ph["table_index"]) * 1e-3),
        "fp32_recheck": {"value": f32["edges_per_s"], "ms_per_step": 1e3 * f32["s_per_step"],
                         "rechecks": f32["rechecks"], "recheck_fraction": f32["rechecks"] / max(1, f32["candidates"]),
                         "identical_to_fp64": res.get("fp32_identical_to_fp64"), "phases_ms": f32["phases_ms"]},
        "roofline": roof,
        # the whole step against the HBM roofline: 172 B per point + 8 B per edge of algorithmic bytes
        "step_roofline": {"bound": "hbm", "algorithmic_bytes": step_bytes(n, f64["m"]),
                          "ms_per_step": 1e3 * f64["s_per_step"], "device_ms": ph["device_total"],
                          "frac": step_bytes(n, f64["m"]) / f64["s_per_step"] / 1e9 / HBM_PEAK_GBS,
                          "roofline_ms": step_bytes(n, f64["m"]) / (HBM_PEAK_GBS * 1e9) * 1e3},
    }
    if serving is not None:
        line["serving"] = serving
    if not args.no_configs:
        line["configs"] = run_configs(args)
    if not args.no_ablation:
        line["fp32_ablation"] = run_ablation(args)
    if not args.no_soft:
        line["soft"] = run_soft(args)
    if args.shares > 1:
        line["share"] = run_shares(args)
    if not args.no_dynamic:
        line["dynamic"] = run_dynamic(args)
    if not args.no_csr:
        line["csr"] = run_csr(args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args, f64["m"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

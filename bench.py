"""Benchmark of the overset grid-assembly hot path on one MI355X.

A step is one pass of the whole path over one time step of the workload:
hole cut, fringe marking + ordered compaction, query transform, donor
search and interpolation of u, v, w, p. Inputs (grids, fields, the pose
table of every step) are resident in HBM before timing starts.

Prints one JSON line. `value` = fringe points assembled and interpolated per
second = sum of per-step query counts / wall time of the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fringe points assembled+interpolated/s per step; mixed-batched vs plain FP64"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(w, budget_s: float) -> dict:
    """The CPU oracle, untuned, on a bounded sample of the same workload:
    whole steps (all five stages) from step 0 on, until `budget_s` of work."""
    import oracle
    o = oracle.Oracle(w.grids, w.nf)
    for g in range(w.ngrids):
        o.bins(g)  # control cells are set-up, not per-step work
    pts, el, steps = 0, 0.0, 0
    while el < budget_s and steps < w.steps:
        t0 = time.perf_counter()
        r = o.step(w.poses[steps], w.fields)
        el += time.perf_counter() - t0
        pts += len(r["q_grid"])
        steps += 1
    return {"value": pts / el, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{w.name} steps 0..{steps - 1} ({steps} full steps, {pts} queries, {el:.1f} s), "
                      f"control cells built beforehand; host CPU {cpu_model()}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C1")
    ap.add_argument("--precision", default=None, help="fp64 or mixed (default: the config's)")
    ap.add_argument("--graph", action="store_true", help="replay each step from a captured HIP graph")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this path has no multi-GPU form.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_1910_09315_amd.assembly import Assembly

    t0 = time.perf_counter()
    w = W.build(args.config)
    precision = args.precision or w.precision
    log(f"[bench] workload {w.name} built in {time.perf_counter() - t0:.1f}s: {w.total_nodes} nodes, "
        f"{w.ngrids} grids, {w.steps} poses, precision {precision}")
    dev = torch.device("cuda", 0)
    a = Assembly(w.grids, w.nf, fields=w.fields, precision=precision)
    n0 = a.count_queries(w.poses[0])
    a.allocate(2 * n0 + 4096)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).to(dev)
    log(f"[bench] set-up done, {n0} queries at t=0, capacity {a.capacity}")
    if args.graph:
        a.capture()
        run = lambda t: a.replay(poses[t % w.steps])
    else:
        run = lambda t: a.step(poses[t % w.steps])

    for t in range(args.warmup):
        run(t)
    torch.cuda.synchronize(dev)
    log("[bench] warm-up done")

    # timed region: K steps; per-step query counts accumulate on the device
    counts = torch.zeros(args.steps, dtype=torch.int64, device=dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    hc = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    from paper_1910_09315_amd import binding as B
    torch.cuda.synchronize(dev)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    start.record()
    for k in range(args.steps):
        t = args.warmup + k
        ev[k][0].record()
        if args.graph:
            run(t)
        else:
            p = poses[t % w.steps]
            cap = a.capacity
            hc[k][0].record()
            B.overset_holecut(a.ctx, p, a.flags)
            hc[k][1].record()
            B.overset_fringe_compact(a.ctx, a.nf, a.flags, a.q_grid, a.q_node, cap, a.d_count)
            B.overset_transform(a.ctx, p, a.q_grid, a.q_node, a.d_count, cap, a.qx)
            B.overset_donor_search(a.ctx, p, a.flags, a.q_grid, a.q_node, a.qx, a.d_count, cap, a.donor_grid,
                                   a.donor_cell, a.s, a.status)
            B.overset_interp(a.ctx, a.donor_grid, a.donor_cell, a.s, a.d_count, cap, a.fields, a.out)
        ev[k][1].record()
        counts[k:k + 1].copy_(a.d_count, non_blocking=True)
    stop.record()
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    status = a.ctx.status()
    queries = int(counts.sum().item())
    step_ms = np.array([e[0].elapsed_time(e[1]) for e in ev])
    value = queries / (total_ms / 1e3)
    log(f"[bench] {args.steps} steps: {total_ms:.2f} ms (wall {wall * 1e3:.1f} ms), {queries} queries, "
        f"median step {np.median(step_ms):.3f} ms, p90 {np.percentile(step_ms, 90):.3f} ms, status {status}")

    roofline = None
    if not args.graph:
        hc_ms = np.array([e[0].elapsed_time(e[1]) for e in hc])
        nodes = w.total_nodes
        per_node = 25 if precision == "fp64" else 13   # coordinates (3 x 8 or 3 x 4 B) + 1 flag byte
        bytes_launch = per_node * nodes
        avg_s = hc_ms.mean() / 1e3
        achieved = bytes_launch / avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": "k_holecut", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "avg_us": round(hc_ms.mean() * 1e3, 2),
                    "algorithmic_bytes_per_launch": bytes_launch,
                    "per_unit": f"{per_node} B per node x {nodes} nodes"}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total_ms / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.grids[0].dims[0]}x{w.grids[0].dims[1]}x{w.grids[0].dims[2]} "
                               f"curvilinear background + {w.ngrids - 1} overset shell(s), rigid motion, "
                               f"{precision}{', hip graph' if args.graph else ''}",
                   "nodes": w.total_nodes, "queries_per_step_mean": round(queries / args.steps, 1),
                   "median_step_ms": round(float(np.median(step_ms)), 4),
                   "p90_step_ms": round(float(np.percentile(step_ms, 90)), 4)},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

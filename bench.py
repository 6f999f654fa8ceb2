"""Benchmark of the overset grid-assembly hot path on one MI355X.

A step is one pass of the whole path over one time step of the workload:
hole cut, fringe marking + ordered compaction, query transform, donor
search and interpolation of u, v, w, p. Inputs (grids, fields, the pose
table of every step) are resident in HBM before timing starts.

Prints one JSON line. `value` = fringe points assembled and interpolated per
second = sum of per-step query counts / wall time of the timed steps, for the
bench workload (default C1, plain FP64). `forms` adds the same metric for the
largest workload (default C4, `--compare`) in mixed precision (the batched
form) and in plain FP64, measured the same way in the same run, so that the
two precisions are compared on the same grids.
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
FP64_PEAK_TFLOPS = 78.6   # MI355X vector FP64
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32
# Algorithmic flops of the one-kernel back half per unit of work, counted from
# its code (adds, multiplies and divides; an FMA counts 2):
#  per walked cell: trilinear map coefficients from the 8 corners (60) plus
#    the residual, Jacobian and determinant at convergence (114; mixed: + the
#    condition estimate, 50);
#  per Newton iteration: residual and Jacobian (100) and the Cramer solve (54);
#  per fallback-scan candidate: the hull rejection test (290) and the map (60);
#  per query: transform (15), body frame and bin (30), weights and the
#    4-field gather (85).
FLOPS_PER_CELL = {"fp64": 174, "mixed": 224}
FLOPS_PER_NEWTON_ITER = 154
FLOPS_PER_SCAN_CANDIDATE = 350
FLOPS_PER_QUERY = 130
KERNEL_SOURCES = ["paper_1910_09315_amd/csrc/ov_search.hip", "paper_1910_09315_amd/csrc/ov_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# work counters (binding.STAT), by index
ST_HC_NODES, ST_HC_CALLS, ST_CELLS, ST_ITERS, ST_CANDS, ST_BACK, ST_FLAG_W, ST_BASE_R, ST_STARTS = range(9)
# Algorithmic HBM bytes of the one-kernel back half (transform + donor search +
# interpolation), per unit, from the per-unit figures of the path's work:
#  per query: its grid and node ids (8) and FP64 node coordinates (24) read;
#    offsets, natural coordinates (3 values each), donor grid + cell (8),
#    status (4) and the 4 interpolated values written;
#  per walked cell: 8 corners x 24 B coordinates;
#  per fallback-scan candidate: its id (4) + 8 corners x 24 B;
#  per distinct donor-corner node: its 4 field values (read once).
BACK_BYTES_PER_CELL = 8 * 24
BACK_BYTES_PER_CAND = 4 + 8 * 24


def back_bytes_per_query(es: int) -> int:
    return 8 + 24 + 3 * es + 3 * es + 8 + 4 + 4 * es


def profiler_counting() -> bool:
    """True inside a rocprofv3 counter-collection run (--pmc or counter
    groups), which serialises kernel dispatches."""
    v = os.environ.get("ROCPROF_COUNTER_COLLECTION", "")
    return v.strip().lower() not in ("", "0", "false", "no", "off")


_WORKLOADS = {}


def load_workload(name: str):
    """The seeded workload `name`, built once per process."""
    import workloads as W
    if name not in _WORKLOADS:
        _WORKLOADS[name] = W.build(name)
    return _WORKLOADS[name]


def source_hash(files) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(key: str):
    """HBM bytes per launch measured with rocprofv3 counters for `key`, or
    None if none were recorded or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            e = json.load(fh).get(key)
    except (OSError, ValueError):
        return None
    if not e or e.get("source_sha256") != source_hash(e.get("sources", KERNEL_SOURCES)):
        return None
    return e.get("bytes_per_launch")


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


def cpu_baseline(w, budget_s: float, check=None) -> tuple[dict, dict | None]:
    """The CPU oracle, untuned, on a bounded sample of the same workload:
    whole steps (all five stages) from step 0 on, until `budget_s` of work.
    check = (t, GPU result of step t): afterwards (untimed) the oracle's step
    t is compared with it; the second return value holds the error norms."""
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
    cores = oracle.num_threads()
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    base = {"value": pts / el, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": f"{w.name} steps 0..{steps - 1} ({steps} full steps, {pts} queries, {el:.1f} s), "
                      f"control cells built beforehand; host CPU {cpu_model()}, os.cpu_count() "
                      f"{os.cpu_count()}, affinity mask {affinity} CPUs"}
    # the same steps on one thread, while they fit in half the budget
    one = None
    if cores > 1 and el / steps * cores <= budget_s / 2:
        oracle.set_threads(1)
        p1, e1, s1 = 0, 0.0, 0
        while (s1 == 0 or e1 < budget_s / 2) and s1 < steps:
            t0 = time.perf_counter()
            r = o.step(w.poses[s1], w.fields)
            e1 += time.perf_counter() - t0
            p1 += len(r["q_grid"])
            s1 += 1
        oracle.set_threads(cores)
        one = {"value": round(p1 / e1, 1), "sample": f"steps 0..{s1 - 1} ({s1} steps, {e1:.1f} s)"}
    base["one_thread"] = one
    return base, (error_norms(o.step(w.poses[check[0]], w.fields), check[1], check[0]) if check else None)


def error_norms(ref: dict, gpu: dict, t: int) -> dict:
    """How step t of the timed executor compares with the oracle's: identical
    flags and query lists, the share of identical donors, and the value
    errors over queries with the same donor, relative to each field's
    largest magnitude."""
    import numpy as np
    n = len(ref["q_grid"])
    same_q = gpu["count"] == n and np.array_equal(gpu["q_grid"], ref["q_grid"]) and \
        np.array_equal(gpu["q_node"], ref["q_node"])
    out = {"step": t, "queries": n, "flags_identical": bool(np.array_equal(gpu["flags"], ref["flags"])),
           "queries_identical": bool(same_q)}
    if same_q and n:
        found = ref["donor_grid"] >= 0
        same = found & (gpu["donor_grid"] == ref["donor_grid"]) & (gpu["donor_cell"] == ref["donor_cell"])
        out["orphans_identical"] = bool(np.array_equal(gpu["donor_grid"] < 0, ~found))
        out["donors_identical_frac"] = round(float(same.sum() / max(1, found.sum())), 6)
        if same.any() and "values" in gpu:
            rv, gv = ref["values"][:, same], gpu["values"][:, same]
            scale = np.maximum(np.abs(rv).max(axis=1, keepdims=True), 1e-300)
            e = np.abs(gv - rv) / scale
            out["value_err_max_rel"] = float(f"{e.max():.3e}")
            out["value_err_rms_rel"] = float(f"{np.sqrt(np.mean(e * e)):.3e}")
    return out


def measure_next_rows(a, b, nrhs: int, reps: int, seed: int = 7) -> dict:
    """Times the calls that follow a step on its buffer set `b`: the
    interpolation matrix (ELL-8), its application to nrhs vectors
    interleaved per node, and the velocity-frame rotation. Each call is
    captured `reps` times into a HIP graph whose replay is timed with events
    on the replaying stream (no host gaps between the launches). Algorithmic
    bytes per launch: what each call must read and write once (for the
    application, each distinct column's x values once)."""
    import torch
    from paper_1910_09315_amd import binding as B
    dev = a.dev
    torch.cuda.synchronize(dev)
    n = min(int(b.d_count.item()), b.capacity)
    es = 4 if a.dtype == torch.float32 else 8
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    x = torch.randn((a.total, nrhs), generator=gen, dtype=torch.float64, device=dev).to(a.dtype).contiguous()
    y = torch.empty((b.capacity, nrhs), dtype=a.dtype, device=dev)
    cols = torch.empty((b.capacity, 8), dtype=torch.int32, device=dev)
    vals = torch.empty((b.capacity, 8), dtype=a.dtype, device=dev)
    B.overset_interp_matrix(a.ctx, b.donor_grid, b.donor_cell, b.s, b.d_count, b.capacity, cols, vals)
    torch.cuda.synchronize(dev)
    live = cols[:n]
    distinct = int(torch.unique(live[live >= 0]).numel())
    poses = torch.zeros(a.ngrids * 12, dtype=torch.float64, device=dev)
    poses[0::12] = 1.0
    poses[4::12] = 1.0
    poses[8::12] = 1.0
    out = b.out.clone()
    calls = {
        "interp_apply": lambda: B.overset_interp_apply(a.ctx, cols, vals, b.d_count, b.capacity, x, nrhs, y,
                                                       layout=1),
        "interp_matrix": lambda: B.overset_interp_matrix(a.ctx, b.donor_grid, b.donor_cell, b.s, b.d_count,
                                                         b.capacity, cols, vals),
        # identity poses: the rotation leaves the values as they are, so every launch sees the same data
        "frame_velocity": lambda: B.overset_frame_velocity(a.ctx, poses, b.q_grid, b.donor_grid, b.d_count,
                                                           b.capacity, out),
    }

    def timed(fn):
        s = torch.cuda.Stream(dev)
        s.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream(dev).wait_stream(s)
        torch.cuda.synchronize(dev)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                fn()
        g.replay()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize(dev)
        return e0.elapsed_time(e1) * 1e3 / reps

    us = {k: timed(f) for k, f in calls.items()}
    nbytes = {"interp_apply": n * 8 * (4 + es) + n * nrhs * es + distinct * nrhs * es,
              "interp_matrix": n * (4 + 4 + 3 * es) + n * 8 * (4 + es),
              "frame_velocity": n * (4 + 4) + 2 * n * 3 * es}
    per_unit = {"interp_apply": f"per row 8 x ({4 + es} B index+weight) + {nrhs} x {es} B y; plus {distinct} "
                                f"distinct columns x {nrhs} x {es} B x (vectors interleaved per node)",
                "interp_matrix": f"per row 8 B donor grid+cell + {3 * es} B s read, 8 x ({4 + es} B) written",
                "frame_velocity": f"per row 8 B grids read + 3 x {es} B read and written"}
    res = {"rows": n, "reps": reps, "nrhs": nrhs,
           "timing": "hip events around a graph replay of reps launches, on the replaying stream"}
    for k in calls:
        gbs = nbytes[k] / (us[k] * 1e-6) / 1e9
        res[k] = {"avg_us": round(us[k], 2), "algorithmic_bytes_per_launch": nbytes[k], "achieved_gbs": round(gbs, 1),
                  "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "rows_per_s": round(n / (us[k] * 1e-6), 1),
                  "per_unit": per_unit[k]}
    return res


def back_roofline(stat, queries_per_launch: float, avg_s: float, precision: str, es: int, distinct_nodes,
                  traffic) -> dict:
    """The one-kernel back half against the chip: algorithmic flops per
    launch against the vector peak of its precision, and algorithmic bytes per
    launch against HBM; `bound` is the resource of the larger fraction.
    stat: work counters summed over the launches timed."""
    launches = max(1, stat[ST_BACK])
    cells, iters, cands = stat[ST_CELLS] / launches, stat[ST_ITERS] / launches, stat[ST_CANDS] / launches
    flops = (FLOPS_PER_CELL[precision] * cells + FLOPS_PER_NEWTON_ITER * iters
             + FLOPS_PER_SCAN_CANDIDATE * cands + FLOPS_PER_QUERY * queries_per_launch)
    peak_fl = FP64_PEAK_TFLOPS if precision == "fp64" else FP32_PEAK_TFLOPS
    tflops = flops / avg_s / 1e12
    nbytes = (back_bytes_per_query(es) * queries_per_launch + BACK_BYTES_PER_CELL * cells
              + BACK_BYTES_PER_CAND * cands + 4 * es * (distinct_nodes or 0))
    gbs = nbytes / avg_s / 1e9
    alu = {"achieved": round(tflops, 4), "peak": peak_fl, "unit": "TFLOP/s", "frac": round(tflops / peak_fl, 6),
           "algorithmic_flops_per_launch": round(flops),
           "per_unit": f"{FLOPS_PER_CELL[precision]} x {cells:.0f} walked cells + {FLOPS_PER_NEWTON_ITER} x "
                       f"{iters:.0f} Newton iterations + {FLOPS_PER_SCAN_CANDIDATE} x {cands:.0f} fallback-scan "
                       f"candidates + {FLOPS_PER_QUERY} x {queries_per_launch:.0f} queries per launch (counted by "
                       f"the kernel)",
           "peak_note": "vector FP64 peak" if precision == "fp64" else
                        "vector FP32 peak (the walk and weights run in FP32; FP64 corrections included)"}
    hbm = {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
           "algorithmic_bytes_per_launch": round(nbytes),
           "per_unit": f"{back_bytes_per_query(es)} B x {queries_per_launch:.0f} queries + {BACK_BYTES_PER_CELL} B "
                       f"x {cells:.0f} walked cells + {BACK_BYTES_PER_CAND} B x {cands:.0f} scan candidates + "
                       f"{4 * es} B x {distinct_nodes} distinct donor-corner nodes per launch"}
    top = hbm if hbm["frac"] >= alu["frac"] else alu
    r = {"bound": "hbm" if top is hbm else "alu", "kernel": "k_back (transform + donor search + interpolation)",
         "achieved": top["achieved"], "peak": top["peak"], "unit": top["unit"], "frac": top["frac"],
         "traffic": traffic,
         "traffic_gbs": round(traffic / avg_s / 1e9, 1) if traffic else None,
         "traffic_frac_hbm": round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
         "avg_us": round(avg_s * 1e6, 2), "hbm_view": hbm, "alu_view": alu}
    return r


def holecut_roofline(stat, avg_s: float, precision: str, nsub: int, note: str) -> dict:
    """The hole-cut stage (start of the step's flags + the culled hole cut)
    against HBM, in the bytes it must move: the flag bytes the step's start
    wrote (the previous step's near tiles in the executors, every node in a
    full fill) and the base flags it read, the coordinates and flag of every
    candidate node tested, and the sub-tile spheres."""
    calls = max(1, stat[ST_HC_CALLS])
    coord_b = 24 if precision == "fp64" else 12
    written, base, cand = stat[ST_FLAG_W] / calls, stat[ST_BASE_R] / calls, stat[ST_HC_NODES] / calls
    nbytes = written + base + (coord_b + 1) * cand + 32 * nsub
    gbs = nbytes / avg_s / 1e9
    return {"bound": "hbm", "kernel": "hole-cut stage (k_flag_reset, then k_holecut_list or k_holecut_sub, in the "
                                      "executors)",
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": None, "avg_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": round(nbytes),
            "per_unit": f"1 B x {written:.0f} flag bytes written + 1 B x {base:.0f} base flags read at the step's "
                        f"start ({stat[ST_STARTS] / calls:.2f} starts per call) + {coord_b + 1} B x {cand:.0f} "
                        f"candidate nodes tested + 32 B x {nsub} sub-tile spheres per launch (counted by the kernels)",
            "timing": note}


def measure(args, w=None):
    """Times args.steps steps of workload args.config; returns (the JSON
    fields, the workload)."""
    import numpy as np
    import torch

    from paper_1910_09315_amd import binding as B
    from paper_1910_09315_amd.assembly import Assembly, Pipeline

    t0 = time.perf_counter()
    if w is None:
        w = load_workload(args.config)
    if args.steps is None:
        args.steps = w.steps - args.warmup
    if args.warmup + args.steps > w.steps:
        log(f"[bench] note: steps {args.warmup}..{args.warmup + args.steps - 1} run past the workload's {w.steps} "
            f"poses and wrap around to pose 0 (a jump the warm start does not follow)")
    precision = args.precision or w.precision
    log(f"[bench] workload {w.name} ready in {time.perf_counter() - t0:.1f}s: {w.total_nodes} nodes, "
        f"{w.ngrids} grids, {w.steps} poses, precision {precision}")
    dev = torch.device("cuda", 0)
    opts = {"holecut_cull": 0 if args.no_cull else 1}
    if args.npl:
        opts["holecut_npl"] = args.npl
    if args.unfused_back:
        opts["back_fused"] = 0
    if args.max_walk:
        opts["max_walk"] = args.max_walk
    opts["field_layout"] = 1 if args.fields == "interleaved" else 0
    a = Assembly(w.grids, w.nf, fields=w.fields, precision=precision, options=opts)
    n0 = a.count_queries(w.poses[0])
    cap = 2 * n0 + 4096
    a.allocate(cap)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).to(dev)
    tuned = None
    if not (args.graph or args.sequential or args.eager or args.graphs or args.no_tuned):
        from paper_1910_09315_amd import autotune as AT
        sig = AT.signature(w, precision)
        tuned = AT.load(sig)
        if tuned is None and args.autotune:
            t1 = time.perf_counter()
            tuned = AT.tune(a, cap, poses, steps=min(30, w.steps - 3), log=log)
            tuned["workload"] = w.name
            AT.store(sig, tuned)
            log(f"[bench] tuned in {time.perf_counter() - t1:.1f}s: {tuned}")
        if tuned is not None:
            params = dict(tuned["params"])
            if args.npl:
                params["holecut_npl"] = args.npl
            AT.apply(a, params)
            if args.stages is None:
                args.stages = params["stages"]
            if args.threads is None:
                args.threads = int(params.get("threads", 0))
            if args.by_step is None:
                args.by_step = int(params.get("by_step", 0))
            log(f"[bench] tuned parameters {params}")
    for kv in args.opt:
        k, v = kv.split("=", 1)
        a.set_option(k, int(v))
        log(f"[bench] option {k} = {v}")
    if args.stages is None:
        args.stages = 3
    if args.threads is None:
        args.threads = 0
    if args.by_step is None:
        args.by_step = 0
    if args.stages > 1 and profiler_counting():
        # counter collection serialises dispatches: a stream waiting on
        # another stream's counter could wait for work that cannot start
        log(f"[bench] rocprofv3 counter collection detected: the executor runs on one stream "
            f"(asked for {args.stages})")
        args.stages = 1
    mode = ("graph" if args.graph else "sequential" if args.sequential else "pipelined-py" if args.eager else
            "pipelined-graph" if args.graphs else "pipelined")
    log(f"[bench] set-up done, {n0} queries at t=0, capacity {cap}, mode {mode}")
    pipe = None
    max_timed = max(args.steps, 64)
    if mode.startswith("pipelined"):
        pipe = Pipeline(a, cap, native=(mode == "pipelined"), max_timed=max_timed,
                        stages=args.stages if mode == "pipelined" else 2,
                        graphs=(mode == "pipelined" and args.native_graphs),
                        threads=(mode == "pipelined" and bool(args.threads)),
                        by_step=(mode == "pipelined" and bool(args.by_step) and args.stages > 1
                                 and not args.native_graphs))
    elif mode == "graph":
        a.capture()
    if mode == "pipelined-graph":
        pipe.capture()

    counts = torch.zeros(args.steps + args.warmup, dtype=torch.int64, device=dev)
    hc = [] if mode == "graph" else [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                                     for _ in range(args.steps)]

    def run(t, k=None):
        p = poses[t % w.steps]
        cnt = counts[t:t + 1]
        ev = hc[k] if (k is not None and hc) else None
        if pipe is not None:
            pipe.submit(t, p, count_out=cnt, holecut_events=ev)
        elif mode == "graph":
            a.replay(p)
            cnt.copy_(a.d_count, non_blocking=True)
        else:
            if ev is not None:
                ev[0].record()
            B.overset_holecut(a.ctx, p, a.flags)
            if ev is not None:
                ev[1].record()
            B.overset_fringe_compact(a.ctx, a.nf, a.flags, a.q_grid, a.q_node, cap, a.d_count)
            a.back(p, a.buf)
            cnt.copy_(a.d_count, non_blocking=True)

    # the native executor takes the timed steps in one call: their poses as one
    # contiguous device table, prepared before the timed region
    native = pipe is not None and pipe.native is not None
    many = native and not args.per_step_submit
    if many:
        idx = torch.arange(args.warmup, args.warmup + args.steps, device=dev) % w.steps
        timed_poses = poses[idx].contiguous()
    for t in range(args.warmup):
        run(t)
    if pipe is not None:
        pipe.join()
    torch.cuda.synchronize(dev)
    a.ctx.stats()  # zero the work counters: count the timed steps only
    log("[bench] warm-up done")

    # the back half of every time_every-th timed step (from the first) is
    # timed with events on its stream, in place in the pipeline
    roof_back = args.roofline == "back" and native and not args.unfused_back and args.time_every > 0
    if roof_back:
        pipe.native.stage_times(0)  # restart the timing record
        pipe.native.set_timing(args.time_every, 2, alone=False)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    # stream order and argument views are set up before the timed region
    # (the device is idle here, so the order is a formality, not step work)
    if pipe is not None:
        pipe.wait_current()
    timed_counts = counts[args.warmup:args.warmup + args.steps]
    t_wall = time.perf_counter()
    start.record()
    t_host0 = time.perf_counter()
    if many:
        pipe.submit_many(args.warmup, timed_poses, timed_counts)
    else:
        for k in range(args.steps):
            run(args.warmup + k, None if mode == "graph" else k)
    host_ms = (time.perf_counter() - t_host0) * 1e3
    if pipe is not None:
        pipe.join()
    stop.record()
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    status = a.ctx.status()
    stat = a.ctx.stats()
    ntiles = sum(-(-g.dims[0] // 64) * -(-g.dims[1] // 8) * -(-g.dims[2] // 8) for g in w.grids)
    nsub = 4 * ntiles
    queries = int(counts[args.warmup:].sum().item())
    value = queries / (total_ms / 1e3)
    log(f"[bench] {args.steps} steps: {total_ms:.2f} ms (wall {wall * 1e3:.1f} ms, host submit {host_ms:.1f} ms), "
        f"{queries} queries, {total_ms / args.steps * 1e3:.1f} us/step, status {status}")
    es = 4 if precision == "mixed" else 8
    last_t = args.warmup + args.steps - 1
    # the last timed step's results, for the oracle comparison (its pose is
    # the next after the previous step's: the warm start followed the motion)
    last_result = (last_t % w.steps, pipe.results(last_t) if pipe is not None else a.results())

    def distinct_corner_nodes(b):
        """Distinct donor-corner nodes of a step's donors (the interpolation
        matrix's columns), counted on the device."""
        cols = torch.empty((b.capacity, 8), dtype=torch.int32, device=dev)
        vals = torch.empty((b.capacity, 8), dtype=a.dtype, device=dev)
        B.overset_interp_matrix(a.ctx, b.donor_grid, b.donor_cell, b.s, b.d_count, b.capacity, cols, vals)
        n = min(int(b.d_count.item()), b.capacity)
        live = cols[:n]
        return int(torch.unique(live[live >= 0]).numel())

    last_buf = pipe.bufs[last_t % pipe.nsets] if pipe is not None else a.buf
    distinct = distinct_corner_nodes(last_buf)

    roofline = None
    if roof_back:
        pipe.native.set_timing(0)
        ms = np.array(pipe.native.stage_times(max_timed))
        if len(ms):
            traffic = recorded_traffic(f"k_back|{w.name}|{precision}")
            roofline = back_roofline(stat, queries / args.steps, ms.mean() / 1e3, precision, es, distinct, traffic)
            roofline["samples_us"] = [round(x * 1e3, 1) for x in ms]
            roofline["timing"] = (f"hip events on the back half's stream around k_back of every "
                                  f"{args.time_every}-th timed step from the first ({len(ms)} samples), in place in "
                                  f"the pipeline (no extra waits), recorded by the native executor; work counters "
                                  f"summed over the timed steps; distinct corner nodes of the last timed step")
        else:
            log("[bench] warning: no back-half timing samples")
    elif hc and args.roofline != "none" and mode != "graph":
        ms = np.array([e[0].elapsed_time(e[1]) for e in hc])
        roofline = holecut_roofline(stat, ms.mean() / 1e3, precision, nsub,
                                    "hip events around every hole cut of the timed steps (on the stream it runs on)")

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total_ms / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.grids[0].dims[0]}x{w.grids[0].dims[1]}x{w.grids[0].dims[2]} "
                               f"curvilinear background + {w.ngrids - 1} overset shell(s), rigid motion, "
                               f"{precision}, {mode}",
                   "nodes": w.total_nodes, "queries_per_step_mean": round(queries / args.steps, 1),
                   "fields": "u, v, w, p interleaved per node" if args.fields == "interleaved" else
                             "u, v, w, p as four blocks",
                   "mode": mode + (f", native executor on {args.stages} stream(s)"
                                   + (", per-stream graphs" if args.native_graphs else "")
                                   + (", all stages of step t on stream t mod streams"
                                      if args.by_step and args.stages > 1 and not args.native_graphs else
                                      ", one host thread per stream" if args.threads and args.stages > 1 else "")
                                   + (", unfused back half" if args.unfused_back else ", fused back half")
                                   + ("" if args.per_step_submit else ", one submit call for all timed steps")
                                   if mode == "pipelined" else ""),
                   "tuned": tuned["params"] if tuned else None},
        "roofline": roofline,
    }
    if args.next_rows:
        out["next_rows"] = measure_next_rows(a, last_buf, args.apply_nrhs, reps=50)
        log(f"[bench] next rows: {out['next_rows']}")
    if native and args.step_report:
        out["step_report"] = step_report(pipe, a, poses, w, args.warmup + args.steps, min(48, args.steps), dev,
                                         precision, es, nsub, distinct)
        rh = out["step_report"].pop("_holecut_roofline", None)
        if rh is not None:
            out["roofline_holecut"] = rh
        log(f"[bench] step report: {out['step_report']}")
    out["_last_result"] = last_result
    if pipe is not None:
        pipe.close()
    a.close()
    del pipe, a
    torch.cuda.synchronize(dev)
    torch.cuda.empty_cache()
    return out, w


def step_report(pipe, a, poses, w, t0: int, n: int, dev, precision: str, es: int, nsub: int, distinct) -> dict:
    """Untimed, after the measured steps: 3 x n more steps through the same
    executor, with hip events (recorded by the executor on the stream each
    stage runs on) around one stage of every step in turn, for the median
    and p90 of each stage's duration on its own and the work counters of
    those steps; n more steps for the median and p90 of the step interval;
    then the outcome mix of the last step (walk, fallback scan, FP64
    correction, orphan)."""
    import numpy as np
    import torch
    rep = {"steps_per_stage": n, "timing": "hip events around one stage of every step, on its stream; while a "
                                         "stage is timed the executor holds the other stages back, so each "
                                         "duration is that stage alone"}
    names = ("hole_cut", "fringe_compact", "back_half")
    counts = torch.zeros(n, dtype=torch.int64, device=dev)
    t = t0
    for st, name in enumerate(names):
        idx = torch.arange(t, t + n, device=dev) % w.steps
        pp = poses[idx].contiguous()
        torch.cuda.synchronize(dev)
        pipe.native.stage_times(0)
        a.ctx.stats()
        pipe.native.set_timing(1, st, alone=True)
        pipe.submit_many(t, pp, counts)
        pipe.join()
        torch.cuda.synchronize(dev)
        pipe.native.set_timing(0)
        stat = a.ctx.stats()
        ms = np.array(pipe.native.stage_times(n))
        us = ms * 1e3
        rep[name] = {"median_us": round(float(np.median(us)), 2), "p90_us": round(float(np.percentile(us, 90)), 2)}
        if st == 0:
            rep["_holecut_roofline"] = holecut_roofline(
                stat, ms.mean() / 1e3, precision, nsub,
                f"hip events around the hole-cut stage of each of {n} steps after the timed region, run alone "
                f"(recorded by the native executor on its stream); work counters of those steps")
        if st == 2:
            q = float(counts.sum().item()) / n
            r = back_roofline(stat, q, ms.mean() / 1e3, precision, es, distinct, None)
            rep[name]["alone_frac"] = {"hbm": r["hbm_view"]["frac"], "alu": r["alu_view"]["frac"],
                                       "avg_us": r["avg_us"]}
        t += n
    # the step interval: an event on the last stream after each step's back
    # half; consecutive events are one step apart in the steady state
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    torch.cuda.synchronize(dev)
    for i in range(n):
        pipe.submit(t + i, poses[(t + i) % w.steps])
        evs[i].record(pipe.back_stream(t + i))
    pipe.join()
    torch.cuda.synchronize(dev)
    gaps = np.array([evs[i - 1].elapsed_time(evs[i]) for i in range(2, n)]) * 1e3
    rep["step_interval"] = {"median_us": round(float(np.median(gaps)), 2),
                            "p90_us": round(float(np.percentile(gaps, 90)), 2),
                            "timing": "hip events after each step's back half on its stream, steps submitted one "
                                      "call each (the timed run submits all its steps in one call)"}
    t += n
    last = t - 1
    r = pipe.results(last)
    st = r["status"]
    kind = st & 3
    m = max(1, len(st))
    # cells each query's walk visited (status bits 8-15), and the largest of
    # each run of 64 consecutive queries (a wavefront walks as long as its
    # longest walk)
    vis = ((st >> 8) & 255).astype(np.float64)
    nw = len(vis) // 64
    rep["outcomes_last_step"] = {
        "step": last % w.steps, "queries": int(len(st)),
        "walk_frac": round(float(np.sum(kind == 1)) / m, 6),
        "fallback_scan_frac": round(float(np.sum(kind == 2)) / m, 6),
        "orphan_frac": round(float(np.sum(kind == 0)) / m, 6),
        "fp64_fixed_frac": round(float(np.sum((st & 4) != 0)) / m, 6),
        "walk_cells_mean": round(float(vis.mean()), 3) if len(vis) else 0.0,
        "walk_cells_max_per_64_mean": round(float(vis[:nw * 64].reshape(nw, 64).max(axis=1).mean()), 3)
        if nw else 0.0}
    return rep


def oracle_check(w, check, budget_note: str = "") -> dict:
    """The oracle's step check[0] compared with the GPU's (check[1])."""
    import oracle
    t1 = time.perf_counter()
    o = oracle.Oracle(w.grids, w.nf)
    ref = o.step(w.poses[check[0]], w.fields)
    e = error_norms(ref, check[1], check[0])
    e["oracle_s"] = round(time.perf_counter() - t1, 1)
    return e


def sampled_steps(steps: int, every: int) -> list:
    """Indices of the timed steps whose back half the executor times (the
    first timed step, then every `every`-th)."""
    return list(range(0, steps, every)) if every > 0 else []


def make_parser():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: every step of the workload after the warm-up)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C1")
    ap.add_argument("--precision", default=None, help="fp64 or mixed (default: the config's)")
    ap.add_argument("--graph", action="store_true", help="single stream, each step replayed from a HIP graph")
    ap.add_argument("--sequential", action="store_true", help="single stream, eager launches")
    ap.add_argument("--eager", action="store_true", help="two-stream pipeline driven from Python, eager launches")
    ap.add_argument("--graphs", action="store_true", help="two-stream pipeline driven from Python, per-half graphs")
    ap.add_argument("--no-cull", action="store_true", help="hole cut streams every node (no tile culling)")
    ap.add_argument("--stages", type=int, default=None, choices=(1, 2, 3),
                    help="native executor streams (default: the tuned choice, else 3; 1 under rocprofv3 counters)")
    ap.add_argument("--threads", type=int, default=None, choices=(0, 1),
                    help="native executor: one host thread per stream in multi-step submits (default: tuned, else 0)")
    ap.add_argument("--by-step", type=int, default=None, choices=(0, 1),
                    help="native executor, two or three streams: all stages of step t on stream t mod streams "
                         "(default: tuned, else 0)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the executor for this workload first when no tuned entry is cached")
    ap.add_argument("--no-tuned", action="store_true", help="ignore the cached tuned parameters")
    ap.add_argument("--per-step-submit", action="store_true",
                    help="native pipeline: one host call per step instead of one call for all timed steps")
    ap.add_argument("--native-graphs", action="store_true",
                    help="the native executor replays per-stream HIP graphs instead of launching kernels directly")
    ap.add_argument("--fields", choices=("interleaved", "blocks"), default="interleaved",
                    help="field layout in HBM: u, v, w, p interleaved per node, or four blocks")
    ap.add_argument("--max-walk", type=int, default=0, help="walk steps before the fallback scan (0: library default)")
    ap.add_argument("--unfused-back", action="store_true",
                    help="native executor: transform, search and interpolation as separate kernels")
    ap.add_argument("--opt", action="append", default=[], metavar="KEY=VALUE",
                    help="a context option (binding.OPT name) set after the tuned parameters; repeatable")
    ap.add_argument("--npl", type=int, default=0, choices=(0, 4, 16),
                    help="candidate hole-cut nodes per lane (0: the tuned or default choice)")
    ap.add_argument("--time-every", type=int, default=4,
                    help="native executor: time k_back of every N-th timed step from the first with events, in "
                         "place in the pipeline (0: no timing in the timed region)")
    ap.add_argument("--compare", default="C4",
                    help="also time this workload in mixed precision (the batched form) and in FP64 ('' to skip)")
    ap.add_argument("--no-graph-form", dest="graph_form", action="store_false",
                    help="skip timing the main workload with the executor replaying per-stream HIP graphs")
    ap.add_argument("--compare-precisions", default="mixed,fp64",
                    help="precisions of the compared workload, comma-separated")
    ap.add_argument("--roofline", choices=("back", "holecut", "none"), default="back",
                    help="kernel for the roofline object: the one-kernel back half (native executor) or the hole cut")
    ap.add_argument("--no-next-rows", dest="next_rows", action="store_false",
                    help="skip timing the interpolation matrix, its application and the frame rotation")
    ap.add_argument("--apply-nrhs", type=int, default=4, help="vectors per application of the interpolation matrix")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip comparing the last timed step of each workload with the oracle's")
    ap.add_argument("--no-step-report", dest="step_report", action="store_false",
                    help="skip the per-stage durations and outcome mix measured after the timed steps")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB 5 times (reference for HBM counters)")
    return ap


def main():
    args = make_parser().parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / 5
        print(json.dumps({"copy_mib": args.copy_calibration, "bytes_read": n * 8, "bytes_written": n * 8,
                          "avg_ms": round(ms, 4), "gbs_read_plus_write": round(2 * n * 8 / ms / 1e6, 1)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this path has no multi-GPU form.",
              file=sys.stderr)
        sys.exit(2)

    out, w = measure(args)
    last_result = out.pop("_last_result", None)
    if not args.no_oracle_check and last_result is not None:
        log("[bench] comparing the last timed step with the oracle")
        out["vs_oracle"] = oracle_check(w, last_result)
        log(f"[bench] vs oracle: {out['vs_oracle']}")
    import copy
    if args.graph_form and not (args.graph or args.sequential or args.eager or args.graphs or args.native_graphs):
        # the same executor with each stream's stages replayed from HIP graphs
        # captured once per buffer set: host cost per step against direct launches
        a3 = copy.copy(args)
        a3.native_graphs, a3.step_report, a3.next_rows, a3.roofline = True, False, False, "none"
        a3.steps = out["steps"]
        o3, _ = measure(a3, w)
        o3.pop("_last_result", None)
        out.setdefault("forms", {})["native_graphs"] = {
            "workload": o3["config"]["workload"], "value": o3["value"], "ms_per_step": o3["ms_per_step"],
            "over_direct_launches": round(o3["value"] / out["value"], 3),
            "note": "the native executor replaying one HIP graph per stream and step (captured per buffer set; "
                    "each step then starts from a full flag fill, as captured launches cannot alternate near lists)"}
    if args.compare and args.compare != args.config:
        forms = {"note": "the same metric, the value above being the plain FP64 form on its workload; "
                         "`same_workload` times the compared workload in each precision in this run"}
        w2, res = None, {}
        for prec in [p for p in args.compare_precisions.split(",") if p]:
            a2 = copy.copy(args)
            a2.config, a2.precision, a2.steps, a2.stages, a2.max_walk = args.compare, prec, None, None, 0
            a2.threads = None
            a2.by_step = None
            a2.opt = []
            a2.roofline = "back"
            a2.next_rows = args.next_rows and prec == "mixed"
            o2, w2 = measure(a2, w2)
            lr = o2.pop("_last_result", None)
            if not args.no_oracle_check and lr is not None:
                log(f"[bench] comparing the last timed step of {args.compare} ({prec}) with the oracle")
                o2["vs_oracle"] = oracle_check(w2, lr)
                log(f"[bench] vs oracle: {o2['vs_oracle']}")
            res[prec] = {"workload": o2["config"]["workload"], "value": o2["value"],
                         "ms_per_step": o2["ms_per_step"], "steps": o2["steps"],
                         "queries_per_step_mean": o2["config"]["queries_per_step_mean"],
                         "tuned": o2["config"]["tuned"], "roofline": o2.get("roofline"),
                         "roofline_holecut": o2.get("roofline_holecut"), "vs_oracle": o2.get("vs_oracle"),
                         "next_rows": o2.get("next_rows"), "step_report": o2.get("step_report")}
            del lr
        forms["plain_fp64"] = {"workload": out["config"]["workload"], "value": out["value"],
                               "ms_per_step": out["ms_per_step"]}
        if "mixed" in res:
            forms["mixed_batched"] = res["mixed"]
        forms["same_workload"] = {p: {"value": r["value"], "ms_per_step": r["ms_per_step"],
                                      "roofline": r["roofline"], "vs_oracle": r["vs_oracle"]}
                                  for p, r in res.items() if p != "mixed"}
        if "mixed" in res and "fp64" in res:
            forms["same_workload"]["workload"] = args.compare
            forms["same_workload"]["mixed_over_fp64"] = round(res["mixed"]["value"] / res["fp64"]["value"], 3)
        out.setdefault("forms", {}).update(forms)
        del w2
        _WORKLOADS.pop(args.compare, None)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"], _ = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

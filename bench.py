"""Benchmark of the overset grid-assembly hot path on one MI355X.

A step is one pass of the whole path over one time step of the workload:
hole cut, fringe marking + ordered compaction, query transform, donor
search and interpolation of u, v, w, p. Inputs (grids, fields, the pose
table of every step) are resident in HBM before timing starts.

Prints one JSON line. `value` = fringe points assembled and interpolated per
second = sum of per-step query counts / wall time of the timed steps, for the
bench workload (default C1, plain FP64). `forms` adds the same metric for the
mixed-precision batched form (default C4, `--compare`), measured the same way
in the same run.
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


def measure(args):
    """Times args.steps steps of workload args.config; returns (the JSON fields, the workload)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1910_09315_amd import binding as B
    from paper_1910_09315_amd.assembly import Assembly, Pipeline

    t0 = time.perf_counter()
    w = W.build(args.config)
    if args.steps is None:
        args.steps = w.steps - args.warmup
    if args.warmup + args.steps > w.steps:
        log(f"[bench] note: steps {args.warmup}..{args.warmup + args.steps - 1} run past the workload's {w.steps} "
            f"poses and wrap around to pose 0 (a jump the warm start does not follow)")
    precision = args.precision or w.precision
    log(f"[bench] workload {w.name} built in {time.perf_counter() - t0:.1f}s: {w.total_nodes} nodes, "
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
            log(f"[bench] tuned parameters {params}")
    if args.stages is None:
        args.stages = 3
    mode = ("graph" if args.graph else "sequential" if args.sequential else "pipelined-py" if args.eager else
            "pipelined-graph" if args.graphs else "pipelined")
    log(f"[bench] set-up done, {n0} queries at t=0, capacity {cap}, mode {mode}")
    pipe = None
    if mode.startswith("pipelined"):
        pipe = Pipeline(a, cap, native=(mode == "pipelined"), max_timed=args.steps,
                        stages=args.stages if mode == "pipelined" else 2,
                        graphs=(mode == "pipelined" and args.native_graphs))
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
    many = pipe is not None and pipe.native is not None and not args.per_step_submit
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

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    start.record()
    t_host0 = time.perf_counter()
    native = pipe is not None and pipe.native is not None
    roof_back = args.roofline == "back" and native and not args.unfused_back
    timing = native and args.roofline != "none"
    if timing:
        pipe.native.stage_times(0)  # restart the timing record
        pipe.native.set_timing(args.time_every, 2 if roof_back else 0)
    if pipe is not None:
        pipe.wait_current()
    if many:
        pipe.submit_many(args.warmup, timed_poses, counts[args.warmup:args.warmup + args.steps])
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
    queries = int(counts[args.warmup:].sum().item())
    value = queries / (total_ms / 1e3)
    log(f"[bench] {args.steps} steps: {total_ms:.2f} ms (wall {wall * 1e3:.1f} ms, host submit {host_ms:.1f} ms), "
        f"{queries} queries, "
        f"{total_ms / args.steps * 1e3:.1f} us/step, status {status}")

    roofline = None
    if timing:
        pipe.native.set_timing(0)
        ms = np.array(pipe.native.stage_times(args.steps))
        roof_note = (f"hip events around the {'back half' if roof_back else 'hole cut'} of every "
                     f"{args.time_every}-th timed step, recorded by the native executor on the stream it runs on")
    elif hc and args.roofline != "none":
        ms = np.array([e[0].elapsed_time(e[1]) for e in hc])
        roof_note = "hip events around every hole cut of the timed steps (on the stream it runs on)"
    else:
        ms = None
    if ms is not None and len(ms) and roof_back:
        launches = max(1, stat[5])
        cells, iters, cands = stat[2] / launches, stat[3] / launches, stat[4] / launches
        qpl = queries / args.steps
        flops = (FLOPS_PER_CELL[precision] * cells + FLOPS_PER_NEWTON_ITER * iters
                 + FLOPS_PER_SCAN_CANDIDATE * cands + FLOPS_PER_QUERY * qpl)
        avg_s = ms.mean() / 1e3
        peak = FP64_PEAK_TFLOPS if precision == "fp64" else FP32_PEAK_TFLOPS
        # HBM bytes per launch from the counter runs (null once the kernel changed)
        traffic = recorded_traffic(f"k_back|{w.name}|{precision}")
        achieved = flops / avg_s / 1e12
        roofline = {"bound": "alu", "kernel": "k_back (transform + donor search + interpolation)",
                    "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 6),
                    "traffic": traffic,
                    "traffic_gbs": round(traffic / avg_s / 1e9, 1) if traffic else None,
                    "traffic_frac_hbm": round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                    "avg_us": round(ms.mean() * 1e3, 2), "samples_us": [round(x * 1e3, 1) for x in ms],
                    "algorithmic_flops_per_launch": round(flops),
                    "per_unit": f"{FLOPS_PER_CELL[precision]} x {cells:.0f} walked cells + {FLOPS_PER_NEWTON_ITER} "
                                f"x {iters:.0f} Newton iterations + {FLOPS_PER_SCAN_CANDIDATE} x {cands:.0f} "
                                f"fallback-scan candidates + {FLOPS_PER_QUERY} x {qpl:.0f} queries per launch "
                                f"(counted by the kernel)",
                    "peak_note": "vector FP64 peak" if precision == "fp64" else
                                 "vector FP32 peak (the walk and weights run in FP32; FP64 corrections included)",
                    "timing": roof_note}
    elif ms is not None and len(ms):
        nodes = w.total_nodes
        per_node = 25 if precision == "fp64" else 13   # coordinates (3 x 8 or 3 x 4 B) + 1 flag byte
        bytes_launch = per_node * nodes
        if not args.no_cull:
            # culled sub-tiles move only their flag byte (grids with outer
            # fringe layers also read it from the precomputed base flags):
            # count the coordinates the kernel actually read, per launch, from
            # the library's counters, and the sub-tile spheres
            coord_b = 24 if precision == "fp64" else 12
            nsub = 4 * ntiles
            base_nodes = sum(g.nodes for g in w.grids if any(g.outer))
            bytes_launch = int(nodes + base_nodes + coord_b * stat[0] / max(1, stat[1]) + 32 * nsub)
            per_node = f"1 B flag written x {nodes} nodes + 1 B base flag read x {base_nodes} nodes + {coord_b} B " \
                       f"coordinates x {stat[0] / max(1, stat[1]):.0f} nodes read + 32 B x {nsub} sub-tile spheres"
        avg_s = ms.mean() / 1e3
        achieved = bytes_launch / avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": "hole cut (k_flag_fill + k_holecut_sub)" if not args.no_cull
                    else "k_holecut", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "avg_us": round(ms.mean() * 1e3, 2),
                    "algorithmic_bytes_per_launch": bytes_launch,
                    "per_unit": per_node if isinstance(per_node, str) else f"{per_node} B per node x {nodes} nodes",
                    "timing": roof_note}

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
                                   + (", unfused back half" if args.unfused_back else ", fused back half")
                                   + ("" if args.per_step_submit else ", one submit call for all timed steps")
                                   if mode == "pipelined" else ""),
                   "tuned": tuned["params"] if tuned else None},
        "roofline": roofline,
    }
    if args.next_rows:
        last = args.warmup + args.steps - 1
        b = pipe.bufs[last % pipe.nsets] if pipe is not None else a.buf
        out["next_rows"] = measure_next_rows(a, b, args.apply_nrhs, reps=50)
        log(f"[bench] next rows: {out['next_rows']}")
    if native and args.step_report:
        out["step_report"], last_result = step_report(pipe, poses, w, args.warmup + args.steps,
                                                      min(48, args.steps), dev)
        log(f"[bench] step report: {out['step_report']}")
        out["_last_result"] = last_result
    return out, w


def step_report(pipe, poses, w, t0: int, n: int, dev):
    """Untimed, after the measured steps: 3 x n more steps through the same
    executor, with hip events (recorded by the executor on the stream each
    stage runs on) around one stage of every step in turn, for the median
    and p90 of each stage's duration on its own; n more steps for the
    median and p90 of the step interval; then the outcome mix of the last
    step (walk, fallback scan, FP64 correction, orphan)."""
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
        pipe.native.set_timing(1, st)
        pipe.submit_many(t, pp, counts)
        pipe.join()
        torch.cuda.synchronize(dev)
        pipe.native.set_timing(0)
        us = np.array(pipe.native.stage_times(n)) * 1e3
        rep[name] = {"median_us": round(float(np.median(us)), 2), "p90_us": round(float(np.percentile(us, 90)), 2)}
        t += n
    # the step interval: an event on the last stream after each step's back
    # half; consecutive events are one step apart in the steady state
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    torch.cuda.synchronize(dev)
    for i in range(n):
        pipe.submit(t + i, poses[(t + i) % w.steps])
        evs[i].record(pipe.streams[-1])
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
    rep["outcomes_last_step"] = {
        "step": last % w.steps, "queries": int(len(st)),
        "walk_frac": round(float(np.sum(kind == 1)) / m, 6),
        "fallback_scan_frac": round(float(np.sum(kind == 2)) / m, 6),
        "orphan_frac": round(float(np.sum(kind == 0)) / m, 6),
        "fp64_fixed_frac": round(float(np.sum((st & 4) != 0)) / m, 6)}
    return rep, (last % w.steps, r)


def main():
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
                    help="native executor streams (default: the tuned choice, else 3)")
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
    ap.add_argument("--npl", type=int, default=0, choices=(0, 4, 16),
                    help="candidate hole-cut nodes per lane (0: the tuned or default choice)")
    ap.add_argument("--time-every", type=int, default=48,
                    help="native executor: time the roofline kernel of every N-th step with events, run alone (the "
                         "executor drains the other streams around it: each sample costs about 1.5 steps)")
    ap.add_argument("--compare", default="C4",
                    help="also time this workload (the mixed-precision batched form) and report both ('' to skip)")
    ap.add_argument("--roofline", choices=("back", "holecut", "none"), default="back",
                    help="kernel for the roofline object: the one-kernel back half (native executor) or the hole cut")
    ap.add_argument("--no-next-rows", dest="next_rows", action="store_false",
                    help="skip timing the interpolation matrix, its application and the frame rotation")
    ap.add_argument("--apply-nrhs", type=int, default=4, help="vectors per application of the interpolation matrix")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-step-report", dest="step_report", action="store_false",
                    help="skip the per-stage durations and outcome mix measured after the timed steps")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB 5 times (reference for HBM counters)")
    args = ap.parse_args()
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
    if args.compare and args.compare != args.config:
        import copy
        import gc
        import torch
        gc.collect()
        torch.cuda.empty_cache()
        a2 = copy.copy(args)
        a2.config, a2.precision, a2.steps, a2.stages, a2.max_walk = args.compare, None, None, None, 0
        a2.roofline = "none"
        o2, w2 = measure(a2)
        o2.pop("_last_result", None)
        out["forms"] = {
            "note": "the same metric for the plain FP64 form (value above) and the mixed-precision batched form",
            "plain_fp64": {"workload": out["config"]["workload"], "value": out["value"],
                           "ms_per_step": out["ms_per_step"]},
            "mixed_batched": {"workload": o2["config"]["workload"], "value": o2["value"],
                              "ms_per_step": o2["ms_per_step"], "steps": o2["steps"],
                              "queries_per_step_mean": o2["config"]["queries_per_step_mean"],
                              "tuned": o2["config"]["tuned"], "next_rows": o2.get("next_rows"),
                              "step_report": o2.get("step_report")},
            "mixed_batched_over_plain_fp64": round(o2["value"] / out["value"], 3)}
        del w2
    last_result = out.pop("_last_result", None)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"], err = cpu_baseline(w, args.cpu_budget, check=last_result)
        if err is not None:
            out["step_report"]["vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Autotuner for the step executor and its kernels.

The tuned parameters and what they choose:
  stages        streams of the native executor (1, 2 or 3): host time per
                step against overlap of the stages on the device;
  threads       a multi-step submit issues each stream's work from a host
                thread of its own (1) or all of it from the calling thread (0);
  by_step       two or three streams: all stages of step t on stream t mod
                streams (1), or stream g running stage group g (0);
  holecut_npl   candidate hole cut, nodes per lane: 4 (one 256-thread block
                per 16x8x8 sub-tile) or 16 (one wavefront per sub-tile);
  persist       workgroups per CU of the persistent front-half kernels
                (candidate hole cut, compaction);
  back_block    threads per workgroup of the one-kernel back half (64, 128,
                256; also the width of its cooperative fallback scan);
  back_blocks   its workgroups per CU;
  max_walk      stencil-walk steps before a query goes to the workgroup's
                cooperative brute-force scan (a long walk is one lane's serial
                chain, which the whole kernel waits for);
  back_fused    the back half as one kernel (1) or two (2: the walk, then
                the FP64 corrections and scans of the queries it left);
  back_queue    the back half's workgroups take their query chunks from an
                atomic work queue (1) or by a fixed stride (0);
  back_xcd      runs of this many consecutive chunks taken by index go to the
                workgroups of one XCD (neighbouring chunks share its L2; 0:
                launch order);
  holecut_list  the sub-tile cull in the kernel that starts the step and the
                candidates handed out one per hole-cut workgroup by rank (1),
                or each hole-cut workgroup culling and testing its own share
                of the sub-tiles (0).
All but max_walk leave the results unchanged (the parity tests run them);
max_walk can change the reported cell only for a point that lies within the
containment tolerance of a face shared by two valid cells (the walk keeps
the first it meets, the scan the lowest index), never for a point with a
margin to every face.

Search: coordinate descent from the library defaults, two passes over the
parameters, each candidate timed over the same steps of the workload (from a
reset warm-start history, after a short warm-up) with events around one
multi-step submit. Results are cached in a JSON file keyed by the device's
architecture and compute-unit count, the precision, the grid dimensions and
the buffer width.
"""
from __future__ import annotations

import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")

SPACE = {
    "stages": (1, 2, 3),
    "threads": (0, 1),
    "by_step": (0, 1),
    "holecut_npl": (4, 16),
    "persist": (4, 8, 16),
    "back_block": (64, 128, 256),
    "back_blocks": (2, 4, 8, 16),
    "max_walk": (8, 16, 32),
    "back_fused": (1, 2),
    "back_queue": (0, 1),
    "back_xcd": (0, 8),
    "holecut_list": (0, 1),
}
DEFAULTS = {"stages": 3, "threads": 0, "by_step": 0, "holecut_npl": 16, "persist": 8, "back_block": 256, "back_blocks": 8, "max_walk": 16,
            "back_fused": 1, "back_queue": 0, "back_xcd": 0, "holecut_list": 0}
CTX_OPTIONS = ("holecut_npl", "persist", "back_block", "back_blocks", "max_walk", "back_fused", "back_queue",
               "back_xcd", "holecut_list")


def signature(w, precision: str) -> str:
    import torch
    if torch.cuda.is_available():
        pr = torch.cuda.get_device_properties(0)
        dev = f"{pr.gcnArchName.split(':')[0]}x{pr.multi_processor_count}"
    else:
        dev = "cpu"
    dims = ";".join("x".join(str(d) for d in g.dims) for g in w.grids)
    return f"{dev}|{precision}|nf{w.nf}|{dims}"


def load(sig: str, path: str = CACHE):
    try:
        with open(path) as fh:
            return json.load(fh).get(sig)
    except (OSError, ValueError):
        return None


def store(sig: str, entry: dict, path: str = CACHE):
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        d = {}
    d[sig] = entry
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
        fh.write("\n")


def time_config(asm, capacity: int, poses, params: dict, steps: int, warmup: int) -> float:
    """Microseconds per step of the native executor with `params`, over
    poses[warmup : warmup + steps] after warm-up steps poses[:warmup], from a
    reset warm-start history."""
    import torch
    from .assembly import Pipeline
    for k in CTX_OPTIONS:
        asm.ctx.set_option(k, params[k])
    asm.ctx.reset_history()
    pipe = Pipeline(asm, capacity, native=True, stages=params["stages"], threads=bool(params.get("threads", 0)),
                    by_step=bool(params.get("by_step", 0)) and params["stages"] > 1)
    pipe.submit_many(0, poses[:warmup])
    pipe.join()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pipe.wait_current()  # (stream order only: the device is idle here)
    timed = poses[warmup:warmup + steps]
    t0.record()
    pipe.submit_many(warmup, timed)
    pipe.join()
    t1.record()
    torch.cuda.synchronize()
    us = t0.elapsed_time(t1) * 1e3 / steps
    pipe.native.close()
    return us


def normalized(p: dict) -> dict:
    """The parameters with those that cannot act at their defaults: no by-step
    order on one stream, one host thread on one stream or in the by-step
    order (which issues every step from the calling thread)."""
    q = dict(p)
    if q.get("stages", 3) == 1:
        q["by_step"] = 0
    if q.get("stages", 3) == 1 or q.get("by_step", 0):
        q["threads"] = 0
    return q


def tune(asm, capacity: int, poses, steps: int = 30, warmup: int = 3, passes: int = 2, log=print,
         start: dict | None = None) -> dict:
    """Coordinate descent over SPACE from `start` (default: the library
    defaults); returns the best parameters with their time per step and the
    number of configurations timed."""
    best = dict(DEFAULTS)
    if start:
        best.update({k: v for k, v in start.items() if k in SPACE})
    best = normalized(best)
    seen = {}

    def cost(p):
        key = tuple(sorted(p.items()))
        if key not in seen:
            seen[key] = time_config(asm, capacity, poses, p, steps, warmup)
            log(f"[autotune] {p} -> {seen[key]:.1f} us/step")
        return seen[key]

    best_us = cost(best)
    for _ in range(passes):
        changed = False
        for name, values in SPACE.items():
            for v in values:
                if v == best[name]:
                    continue
                cand = normalized(dict(best, **{name: v}))
                if cand == best:
                    continue
                us = cost(cand)
                if us < best_us * 0.99:  # a clear gain only
                    best, best_us, changed = cand, us, True
        if not changed:
            break
    for k in CTX_OPTIONS:
        asm.ctx.set_option(k, best[k])
    asm.ctx.reset_history()
    return {"params": best, "us_per_step": round(best_us, 2), "configs_timed": len(seen),
            "steps": steps, "warmup": warmup, "when": time.strftime("%Y-%m-%d")}


def apply(asm, params: dict):
    for k in CTX_OPTIONS:
        if k in params:
            asm.ctx.set_option(k, params[k])


def main():
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import workloads as W
    from .assembly import Assembly
    ap = argparse.ArgumentParser(description="tune the step executor for a workload and cache the result")
    ap.add_argument("--config", default="C1")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--fields", choices=("interleaved", "blocks"), default="interleaved")
    ap.add_argument("--from-cache", action="store_true", help="start the search from the cached entry, if any")
    args = ap.parse_args()
    w = W.build(args.config)
    precision = args.precision or w.precision
    a = Assembly(w.grids, w.nf, fields=w.fields, precision=precision,
                 options={"field_layout": 1 if args.fields == "interleaved" else 0})
    cap = 2 * a.count_queries(w.poses[0]) + 4096
    a.allocate(cap)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    steps = min(args.steps, w.steps - 3)
    sig = signature(w, precision)
    cached = load(sig, args.out) if args.from_cache else None
    res = tune(a, cap, poses, steps=steps, start=cached["params"] if cached else None)
    res["workload"] = w.name
    store(sig, res, args.out)
    print(json.dumps({"signature": sig, **res}), flush=True)


if __name__ == "__main__":
    main()

"""GPU parity on the many-grid workloads: a school of fish-shaped ellipsoidal
shells over a stretched background (overlapping overset grids exchange
fringe points) and many spherical shells with three fringe layers. Small
variants are checked at every step in both precisions; the full-size cases
run through the three-stream native executor with interleaved fields, as the
benchmark does, and are checked at sampled steps. Needs an MI355X."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from parity import compare

pytestmark = pytest.mark.gpu

MIXED = dict(value_rtol=1e-5, s_tol=1e-4, qx_tol=1e-6)
FP64 = dict(value_rtol=1e-12, s_tol=1e-12, qx_tol=1e-14)


def _check(o, w, t, g, precision):
    r = o.step(w.poses[t], w.fields)
    st = compare(o, w.poses[t], r, g, **(FP64 if precision == "fp64" else MIXED))
    st["step"] = t
    # overlapping overset grids give each other donors in these workloads
    ovov = int(np.count_nonzero((r["q_grid"] > 0) & (r["donor_grid"] > 0)))
    st["overset_to_overset"] = ovov
    print(w.name, precision, st, flush=True)
    return st


def _run_steps(w, steps, precision, options=None):
    from paper_1910_09315_amd.assembly import Assembly
    o = oracle.Oracle(w.grids, w.nf)
    a = Assembly(w.grids, w.nf, fields=w.fields, precision=precision, options=options)
    a.allocate(2 * a.count_queries(w.poses[0]) + 1024)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    out = []
    for t in range(max(steps) + 1):
        a.step(poses[t])
        if t in steps:
            out.append(_check(o, w, t, a.results(), precision))
    assert (a.ctx.status() & ~2) == 0
    return out


def _run_pipeline(w, steps, precision, stages=3, options=None, by_step=False):
    from paper_1910_09315_amd.assembly import Assembly, Pipeline
    o = oracle.Oracle(w.grids, w.nf)
    a = Assembly(w.grids, w.nf, fields=w.fields, precision=precision, options=options)
    cap = 2 * a.count_queries(w.poses[0]) + 4096
    a.allocate(cap)
    pipe = Pipeline(a, cap, native=True, stages=stages, by_step=by_step and stages > 1)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    out = []
    for t in range(max(steps) + 1):
        pipe.submit(t, poses[t])
        if t in steps:
            out.append(_check(o, w, t, pipe.results(t), precision))
    pipe.join()
    torch.cuda.synchronize()
    assert (a.ctx.status() & ~2) == 0
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_school_small_every_step(precision):
    w = W.c3_small(steps=6)
    stats = _run_steps(w, list(range(6)), precision)
    assert sum(s["overset_to_overset"] for s in stats) > 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shells_small_every_step(precision):
    w = W.c4_small(steps=5)
    _run_steps(w, list(range(5)), precision)


def test_shells_small_streaming_holecut():
    w = W.c4_small(steps=2)
    _run_steps(w, [0, 1], "mixed", options={"holecut_cull": 0})


def test_school_small_block_candidate_holecut():
    w = W.c3_small(steps=3)
    _run_steps(w, [0, 1, 2], "mixed", options={"holecut_npl": 4})


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_school_small_listed_candidate_holecut(precision):
    w = W.c3_small(steps=3)
    _run_steps(w, [0, 1, 2], precision, options={"holecut_list": 1})


@pytest.mark.timeout(300)
def test_shells_full_size_listed_candidate_holecut():
    """The full-size shells workload with the listed-candidate hole cut through
    the three-stream executor (flags, query list and donors against the
    oracle at sampled steps)."""
    w = W.c4(steps=500)
    stats = _run_pipeline(w, [0, 1, 250], "mixed", options={"field_layout": 1, "holecut_list": 1, "persist": 4})
    assert all(s["orphans"] == 0 for s in stats)


@pytest.mark.timeout(300)
def test_school_full_size_pipelined_sampled_steps():
    w = W.c3(steps=200)
    stats = _run_pipeline(w, [0, 1, 100, 199], "mixed", options={"field_layout": 1})
    assert all(s["orphans"] == 0 for s in stats)
    assert sum(s["overset_to_overset"] for s in stats) > 0


@pytest.mark.timeout(300)
def test_shells_full_size_pipelined_sampled_steps():
    w = W.c4(steps=500)
    stats = _run_pipeline(w, [0, 499], "mixed", options={"field_layout": 1, "max_walk": 8})
    assert all(s["orphans"] == 0 for s in stats)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("config,precision,sample", [("C4", "mixed", [0, 3, 250]), ("C4", "fp64", [0, 3]),
                                                     ("C3", "mixed", [0, 3, 150]), ("C1", "fp64", [0, 3, 60])])
def test_full_size_tuned_parameters(config, precision, sample):
    """Each full-size workload the benchmark times, through the executor with
    the tuned parameters it applies (streams and their order, hole-cut form
    and width, persistence, back-half form, block and workgroups, walk limit,
    chunk order), checked against the oracle."""
    from paper_1910_09315_amd import autotune as AT
    w = W.build(config)
    tuned = AT.load(AT.signature(w, precision))
    assert tuned is not None, "no tuned entry for this workload"
    p = dict(tuned["params"])
    opts = {k: p[k] for k in AT.CTX_OPTIONS if k in p}
    opts["field_layout"] = 1
    stats = _run_pipeline(w, sample, precision, stages=p["stages"], options=opts, by_step=bool(p.get("by_step", 0)))
    assert all(s["orphans"] == 0 for s in stats)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("config,precision,nsteps", [("C1", "fp64", 60), ("C3", "mixed", 36)])
def test_by_step_order_full_size_batches_match_five_calls(config, precision, nsteps):
    """Full-size workloads through the executor in the by-step order, six
    steps per multi-step submit (so that the stages of consecutive steps run
    at once on their streams, the fringe passes and compactions of two steps
    among them), against the five calls step by step: the last three steps of
    every batch (the ones whose buffer sets still hold them) bit for bit."""
    from paper_1910_09315_amd.assembly import Assembly, Pipeline
    w = W.build(config)
    a = Assembly(w.grids, w.nf, fields=w.fields, precision=precision, options={"field_layout": 1})
    cap = 2 * a.count_queries(w.poses[0]) + 4096
    a.allocate(cap)
    b = Assembly(w.grids, w.nf, fields=w.fields, precision=precision, options={"field_layout": 1})
    b.allocate(cap)
    pipe = Pipeline(b, cap, native=True, stages=3, by_step=True)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    seq = {}
    checked = 0
    for t0 in range(0, nsteps, 6):
        for t in range(t0, t0 + 6):
            a.step(poses[t])
            if t >= t0 + 3:
                seq[t] = a.results()
        pipe.submit_many(t0, poses[t0:t0 + 6].contiguous())
        pipe.join()
        for t in range(t0 + 3, t0 + 6):
            r = pipe.results(t)
            for k in ("flags", "q_node", "qx", "donor_grid", "donor_cell", "status", "s", "values"):
                assert np.array_equal(r[k], seq[t][k], equal_nan=True), (t, k)
            checked += 1
    torch.cuda.synchronize()
    assert checked == nsteps // 2
    pipe.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_shells_full_size_split_back_half(precision):
    """The full-size shells workload with the two-kernel back half."""
    w = W.c4(steps=500)
    stats = _run_pipeline(w, [0, 2, 499], precision, options={"field_layout": 1, "back_fused": 2})
    assert all(s["orphans"] == 0 for s in stats)


@pytest.mark.timeout(300)
def test_shells_full_size_work_queue():
    """The full-size shells workload with the back half's work queue."""
    w = W.c4(steps=500)
    stats = _run_pipeline(w, [0, 1, 250], "mixed", options={"field_layout": 1, "back_queue": 1, "back_blocks": 2})
    assert all(s["orphans"] == 0 for s in stats)

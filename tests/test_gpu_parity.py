"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs. Needs an MI355X."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from parity import compare

pytestmark = pytest.mark.gpu


def _assembly(w, precision="fp64", capacity=None, options=None):
    from paper_1910_09315_amd.assembly import Assembly
    a = Assembly(w.grids, w.nf, fields=w.fields, precision=precision, options=options)
    if capacity is None:
        capacity = 2 * a.count_queries(w.poses[0]) + 1024
    a.allocate(capacity)
    return a


def _run_and_compare(w, steps, precision="fp64", value_rtol=1e-12, s_tol=1e-12, options=None):
    qx_tol = 1e-14 if precision == "fp64" else 1e-6
    o = oracle.Oracle(w.grids, w.nf)
    a = _assembly(w, precision, options=options)
    poses_dev = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    stats = []
    for t in range(max(steps) + 1):
        a.step(poses_dev[t])
        if t in steps:
            g = a.results()
            r = o.step(w.poses[t], w.fields)
            st = compare(o, w.poses[t], r, g, value_rtol=value_rtol, s_tol=s_tol, qx_tol=qx_tol)
            st["step"] = t
            print(w.name, precision, st, flush=True)
            stats.append(st)
    assert (a.ctx.status() & ~2) == 0
    return stats


def test_c0_fp64_matches_oracle():
    w = W.c0()
    st = _run_and_compare(w, [0])[0]
    assert st["queries"] == 1040 and st["orphans"] == 144 and st["near"] == 0


def test_c1_small_fp64_matches_oracle_every_step():
    w = W.c1_small(steps=6)
    _run_and_compare(w, list(range(6)))


def test_c1_small_streaming_holecut_matches_oracle():
    """The same step with the culling hole cut switched off (every node streamed)."""
    w = W.c1_small(steps=3)
    _run_and_compare(w, [0, 1, 2], options={"holecut_cull": 0})
    _run_and_compare(w, [0, 2], precision="mixed", value_rtol=1e-5, s_tol=1e-4, options={"holecut_cull": 0})


def test_c1_small_block_candidate_holecut_matches_oracle():
    """The culled hole cut with one block per candidate sub-tile (4 nodes per lane)."""
    w = W.c1_small(steps=3)
    _run_and_compare(w, [0, 1, 2], options={"holecut_npl": 4})
    _run_and_compare(w, [0, 2], precision="mixed", value_rtol=1e-5, s_tol=1e-4, options={"holecut_npl": 4})


def test_c1_small_listed_candidate_holecut_matches_oracle():
    """The culled hole cut with the sub-tile cull done by the kernel that
    starts the step and the candidates handed out one per block by rank."""
    w = W.c1_small(steps=3)
    _run_and_compare(w, [0, 1, 2], options={"holecut_list": 1})
    _run_and_compare(w, [0, 2], precision="mixed", value_rtol=1e-5, s_tol=1e-4, options={"holecut_list": 1})


def test_c1_small_interleaved_fields_match_oracle():
    """Fields interleaved per node (u, v, w, p) instead of four blocks."""
    w = W.c1_small(steps=3)
    _run_and_compare(w, [0, 2], options={"field_layout": 1})
    _run_and_compare(w, [0, 2], precision="mixed", value_rtol=1e-5, s_tol=1e-4, options={"field_layout": 1})


def test_c1_small_mixed_matches_oracle():
    w = W.c1_small(steps=6)
    stats = _run_and_compare(w, list(range(6)), precision="mixed", value_rtol=1e-5, s_tol=1e-4)
    print("mixed value errors", [s["value_err"] for s in stats])


@pytest.fixture(scope="module")
def c1():
    return W.c1(steps=100)


def test_c1_fp64_matches_oracle_sampled_steps(c1):
    _run_and_compare(c1, [0, 1, 2, 50, 99])


def test_c2_mixed_matches_oracle_sampled_steps(c1):
    stats = _run_and_compare(c1, [0, 1, 50, 99], precision="mixed", value_rtol=1e-5, s_tol=1e-4)
    print("C2 value errors", [s["value_err"] for s in stats])


def test_c1_every_query_by_fallback_scan_matches_oracle(c1):
    """max_walk = 1 without warm start sends (nearly) every C1 query to the
    block-cooperative scan of its control cell, through the sub-bin lists of
    the shell's crowded polar control cells."""
    _run_and_compare(c1, [0, 1], options={"max_walk": 1, "warm": 0})


def test_warm_equals_cold_and_runs_are_deterministic():
    w = W.c1_small(steps=4)
    a = _assembly(w)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    warm = []
    for t in range(4):
        a.step(poses[t])
        warm.append(a.results())
    # cold: forget the history before the last step
    a.ctx.reset_history()
    a.step(poses[3])
    cold = a.results()
    o = oracle.Oracle(w.grids, w.nf)
    ref = o.step(w.poses[3], w.fields)
    gated = (ref["donor_grid"] >= 0) & (ref["margin"] >= 1e-3)
    assert np.array_equal(cold["donor_cell"][gated], warm[3]["donor_cell"][gated])
    assert np.array_equal(cold["donor_grid"] < 0, warm[3]["donor_grid"] < 0)
    # a second identical system gives bitwise identical results at every step
    b = _assembly(w, capacity=a.capacity)
    for t in range(4):
        b.step(poses[t])
        r = b.results()
        for k in ("flags", "q_grid", "q_node", "donor_grid", "donor_cell", "status", "s", "values"):
            assert np.array_equal(r[k], warm[t][k], equal_nan=True), (t, k)


def test_max_walk_one_forces_fallback_same_donors():
    w = W.c1_small(steps=2)
    o = oracle.Oracle(w.grids, w.nf)
    a = _assembly(w, options={"max_walk": 1, "warm": 0})
    a.step(w.poses[1])
    g = a.results()
    r = o.step(w.poses[1], w.fields)
    compare(o, w.poses[1], r, g, value_rtol=1e-12)


def test_capacity_overflow_sets_status_and_writes_nothing_past_capacity():
    w = W.c0()
    a = _assembly(w, capacity=100)
    sentinel = torch.full((200,), -7, dtype=torch.int32, device="cuda")
    a.buf.q_grid = torch.cat([a.q_grid[:100], sentinel[:100]]).contiguous()
    a.buf.q_node = torch.cat([a.q_node[:100], sentinel[100:]]).contiguous()
    a.step(w.poses[0])
    torch.cuda.synchronize()
    assert int(a.d_count.item()) == 1040
    assert a.ctx.status() & 1
    assert torch.all(a.q_grid[100:] == -7) and torch.all(a.q_node[100:] == -7)
    # the first 100 entries are the first 100 of the ordered list
    o = oracle.Oracle(w.grids, w.nf)
    r = o.step(w.poses[0], w.fields)
    assert np.array_equal(a.q_node[:100].cpu().numpy(), r["q_node"][:100])


def test_no_fringe_gives_zero_queries():
    bg = W.cartesian_grid(9)
    g1 = W.cartesian_grid(3, lo=(0.3, 0.3, 0.3), hi=(0.6, 0.6, 0.6))
    w = W.Workload("empty", [bg, g1], nf=0, steps=1, poses=np.stack([W.IDENTITY_POSE] * 2)[None],
                   fields=np.zeros((4, bg.nodes + g1.nodes)))
    a = _assembly(w, capacity=16)
    a.step(w.poses[0])
    r = a.results()
    assert r["count"] == 0 and np.all(r["flags"] == 0)


def test_linear_field_reproduced_on_gpu():
    """u = 1 + 2x - 3y + 0.5z on every grid at t=0 positions is interpolated
    exactly (1e-12) at every non-orphan query of step 0."""
    w = W.c1_small(steps=1)
    off = w.node_offsets
    F = np.zeros((4, w.total_nodes))
    for g, grid in enumerate(w.grids):
        x, y, z = W.world_coords(grid, w.poses[0, g])
        F[0, off[g]:off[g + 1]] = W.linear_field(x, y, z)
    w.fields = F
    a = _assembly(w)
    a.step(w.poses[0])
    r = a.results()
    o = oracle.Oracle(w.grids, w.nf)
    from parity import query_world
    xw = query_world(o, w.poses[0], r["q_grid"], r["q_node"])
    ok = r["donor_grid"] >= 0
    want = W.linear_field(xw[:, 0], xw[:, 1], xw[:, 2])
    assert np.abs(r["values"][0][ok] - want[ok]).max() <= 1e-12 * np.abs(want).max()


def test_graph_replay_matches_eager():
    w = W.c1_small(steps=5)
    a = _assembly(w)
    b = _assembly(w, capacity=a.capacity)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    b.capture()
    for t in range(5):
        a.step(poses[t])
        ra = a.results()
        b.replay(poses[t])
        rb = b.results()
        for k in ("flags", "q_node", "donor_grid", "donor_cell", "s", "values"):
            assert np.array_equal(ra[k], rb[k], equal_nan=True), (t, k)


def test_bad_arguments_rejected_before_launch():
    from paper_1910_09315_amd import binding as B
    w = W.c0()
    a = _assembly(w, capacity=16)
    with pytest.raises(B.OversetError):
        B.overset_fringe_compact(a.ctx, 4, a.flags, a.q_grid, a.q_node, 16, a.d_count)
    with pytest.raises(B.OversetError):
        B.overset_holecut(a.ctx, None, a.flags)
    with pytest.raises(B.OversetError):
        a.ctx.set_option("search_block", 100)
    ctx = B.Context(0)
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(B.OversetError):
        ctx.grid_add((1, 2, 4), 0, x, x, x)
    with pytest.raises(B.OversetError):
        B.overset_holecut(ctx, x, a.flags)  # before finalize


@pytest.mark.parametrize("native,stages,graphs,fused,precision", [
    (True, 1, False, True, "fp64"), (True, 1, False, True, "mixed"), (True, 1, True, True, "fp64"),
    (True, 2, False, True, "fp64"), (True, 2, False, False, "fp64"), (False, 2, False, True, "fp64"),
    (True, 3, False, True, "mixed"), (True, 3, False, False, "mixed"), (True, 2, True, True, "mixed"),
    (True, 3, True, True, "fp64"), (True, 1, False, 2, "fp64"), (True, 3, False, 2, "mixed"),
    (True, 3, False, 2, "fp64"), (True, 2, True, 2, "mixed"), (True, 1, False, 2, "mixed")])
def test_pipeline_matches_sequential(native, stages, graphs, fused, precision):
    """Steps run by the executors (one stream; two streams: front half of
    step t+1 beside the back half of step t; three streams: hole cut of t+1,
    fringe of t and back half of t-1 together), driven by the library's
    executor or from Python, with the back half as one kernel or as the
    separate kernels, equal the single-stream five-call steps bitwise,
    including each step's query count."""
    _check_pipeline(native, stages, graphs, precision, {"back_fused": int(fused)})


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_split_back_half_with_every_query_deferred(precision):
    """The two-kernel back half with the walk limited to one cell and no warm
    start: most queries go through the deferral queue to the cooperative
    scans of the second kernel; the executor's steps equal the five calls'
    bitwise and match the oracle."""
    _check_pipeline(True, 3, False, precision, {"back_fused": 2, "max_walk": 1, "warm": 0},
                    seq_options={"max_walk": 1, "warm": 0})
    w = W.c1_small(steps=3)
    o = oracle.Oracle(w.grids, w.nf)
    from paper_1910_09315_amd.assembly import Pipeline
    a = _assembly(w, precision, options={"back_fused": 2, "max_walk": 1, "warm": 0})
    pipe = Pipeline(a, a.capacity, native=True, stages=1)
    tol = dict(value_rtol=1e-12) if precision == "fp64" else dict(value_rtol=1e-5, s_tol=1e-4, qx_tol=1e-6)
    for t in range(3):
        pipe.submit(t, torch.as_tensor(w.poses[t].reshape(-1)).cuda())
        st = compare(o, w.poses[t], o.step(w.poses[t], w.fields), pipe.results(t), **tol)
        print("split, max_walk 1", precision, st, flush=True)
    pipe.close()


@pytest.mark.parametrize("options", [{"back_block": 64, "back_blocks": 2}, {"back_block": 128, "back_blocks": 16},
                                     {"back_block": 256, "back_blocks": 2, "back_xcd": 8},
                                     {"persist": 4, "holecut_npl": 4}, {"persist": 16}, {"field_layout": 1},
                                     {"holecut_list": 1, "persist": 4}, {"holecut_list": 1, "persist": 16},
                                     {"back_fused": 2, "back_block": 64, "back_blocks": 4},
                                     {"back_fused": 2, "back_block": 256, "back_blocks": 8},
                                     {"back_queue": 1, "back_block": 64, "back_blocks": 2},
                                     {"back_queue": 1, "back_fused": 2, "back_block": 128, "back_blocks": 4},
                                     {"back_xcd": 2, "back_block": 128, "back_blocks": 4},
                                     {"back_xcd": 4, "back_queue": 1, "back_block": 64, "back_blocks": 2},
                                     {"back_xcd": 64, "back_block": 64, "back_blocks": 2}])
def test_tuned_variants_match_sequential(options):
    """Every value the autotuner may pick leaves the results unchanged."""
    _check_pipeline(True, 1, False, "fp64", options)
    _check_pipeline(True, 3, False, "mixed", options)


def _check_pipeline(native, stages, graphs, precision, options, seq_options=None, by_step=False):
    from paper_1910_09315_amd.assembly import Pipeline
    w = W.c1_small(steps=7)
    a = _assembly(w, precision, options=seq_options)
    b = _assembly(w, precision, capacity=a.capacity, options=options)
    pipe = Pipeline(b, a.capacity, native=native, stages=stages, graphs=graphs, by_step=by_step)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    counts = torch.full((7,), -1, dtype=torch.int64, device="cuda")
    seq = []
    for t in range(7):
        a.step(poses[t])
        seq.append(a.results())
    lag = 0 if stages == 1 else 1  # one buffer set: a step's results last until the next step
    for t in range(7):
        pipe.submit(t, poses[t], count_out=counts[t:t + 1])
        if t >= lag:
            r = pipe.results(t - lag)
            for k in ("flags", "q_node", "qx", "donor_grid", "donor_cell", "status", "s", "values"):
                assert np.array_equal(r[k], seq[t - lag][k], equal_nan=True), (t - lag, k)
    pipe.join()
    torch.cuda.synchronize()
    assert counts.cpu().tolist() == [r["count"] for r in seq]


@pytest.mark.parametrize("stages,precision", [(3, "fp64"), (2, "mixed"), (3, "mixed")])
def test_threaded_submit_matches_sequential(stages, precision):
    """Multi-step submits with one host thread per stream (and the back half
    timed in place) give the five calls' results bit for bit, across two
    consecutive batches (the buffer sets' near lists and starts carry over)."""
    from paper_1910_09315_amd.assembly import Pipeline
    w = W.c1_small(steps=10)
    a = _assembly(w, precision)
    b = _assembly(w, precision, capacity=a.capacity)
    pipe = Pipeline(b, a.capacity, native=True, stages=stages, threads=True, max_timed=16)
    pipe.native.set_timing(2, 2, alone=False)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    counts = torch.full((10,), -1, dtype=torch.int64, device="cuda")
    seq = []
    for t in range(10):
        a.step(poses[t])
        seq.append(a.results())
    for t0, t1 in ((0, 7), (7, 10)):
        pipe.submit_many(t0, poses[t0:t1].contiguous(), counts[t0:t1])
        pipe.join()
        for t in range(max(t0, t1 - stages), t1):
            r = pipe.results(t)
            for k in ("flags", "q_node", "qx", "donor_grid", "donor_cell", "status", "s", "values"):
                assert np.array_equal(r[k], seq[t][k], equal_nan=True), (t, k)
    torch.cuda.synchronize()
    assert counts.cpu().tolist() == [r["count"] for r in seq]
    times = pipe.native.stage_times(16)
    assert len(times) == 5 and all(x > 0 for x in times)
    pipe.close()


@pytest.mark.parametrize("stages,precision,options", [(2, "fp64", {}), (3, "fp64", {}), (3, "mixed", {}),
                                                       (2, "mixed", {"back_fused": 2}),
                                                       (3, "mixed", {"holecut_list": 1, "back_xcd": 8})])
def test_by_step_order_matches_sequential(stages, precision, options):
    """The executor with all stages of step t on stream t mod streams gives
    the five calls' results bit for bit, step by step."""
    _check_pipeline(True, stages, False, precision, options, by_step=True)


@pytest.mark.parametrize("stages,precision", [(3, "fp64"), (2, "mixed"), (3, "mixed")])
def test_by_step_order_submit_many_and_timing(stages, precision):
    """The by-step order under multi-step submits, a single-step submit
    between them, the back half timed in place and the fringe stage timed
    alone: results equal the five calls' bit for bit, every timed stage
    yields a positive duration."""
    from paper_1910_09315_amd.assembly import Pipeline
    w = W.c1_small(steps=12)
    a = _assembly(w, precision)
    b = _assembly(w, precision, capacity=a.capacity)
    pipe = Pipeline(b, a.capacity, native=True, stages=stages, by_step=True, max_timed=16)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    counts = torch.full((12,), -1, dtype=torch.int64, device="cuda")
    seq = []
    for t in range(12):
        a.step(poses[t])
        seq.append(a.results())
    for t0, t1, stage, alone in ((0, 5, 2, False), (5, 6, 2, False), (6, 12, 1, True)):
        pipe.native.set_timing(1, stage, alone=alone)
        if t1 - t0 == 1:
            pipe.submit(t0, poses[t0], count_out=counts[t0:t1])
        else:
            pipe.submit_many(t0, poses[t0:t1].contiguous(), counts[t0:t1])
        pipe.join()
        for t in range(max(t0, t1 - stages), t1):
            r = pipe.results(t)
            for k in ("flags", "q_node", "qx", "donor_grid", "donor_cell", "status", "s", "values"):
                assert np.array_equal(r[k], seq[t][k], equal_nan=True), (t, k)
        times = pipe.native.stage_times(16)
        assert len(times) == t1 - t0 and all(x > 0 for x in times), times
    torch.cuda.synchronize()
    assert counts.cpu().tolist() == [r["count"] for r in seq]
    pipe.native.set_timing(0)
    pipe.close()


def test_graph_pipeline_matches_sequential():
    """The two-stream pipeline replaying per-half HIP graphs gives the same
    results as single-stream steps, step by step."""
    from paper_1910_09315_amd.assembly import Pipeline
    w = W.c1_small(steps=7)
    a = _assembly(w)
    b = _assembly(w, capacity=a.capacity)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    seq = []
    for t in range(7):
        a.step(poses[t])
        seq.append(a.results())
    pipe = Pipeline(b, a.capacity, native=False)
    pipe.capture()
    b.ctx.reset_history()
    counts = torch.zeros(7, dtype=torch.int64, device="cuda")
    for t in range(7):
        pipe.submit(t, poses[t], count_out=counts[t:t + 1])
        if t >= 1:
            r = pipe.results(t - 1)
            for key in ("flags", "q_node", "donor_grid", "donor_cell", "status", "s", "values"):
                assert np.array_equal(r[key], seq[t - 1][key], equal_nan=True), (t - 1, key)
    pipe.join()
    assert [int(x) for x in counts.cpu()] == [seq[t]["count"] for t in range(7)]


def seam_case():
    """Buffer reach across a periodic seam whose last tile is thin: a
    cylindrical shell with 121 azimuthal nodes (tiles of 8 leave one node in
    the last) and a blank sphere small enough to cut only its node
    (i=2, j=1, k=4). With nf = 3 the buffer wraps to j = 119, two tiles back."""
    bg = W.cartesian_grid(20)
    cyl = W.cylindrical_shell(6, 121, 9, 0.15, 0.35, 0.3, 0.7)
    cyl.outer = (0, 2, 0, 0, 0, 0)
    ball = W.spherical_shell(6, 8, 7, 0.006, 0.03)
    ball.blank_kind = W.BLANK_SPHERE
    ball.blank_prm = (0.006,)
    ball.outer = (0, 1, 0, 0, 0, 0)
    p_cyl = W.pose12(np.eye(3), (0.5, 0.5, 0.0))
    m = 2 + 6 * (1 + 121 * 4)
    centre = np.array([cyl.X[m], cyl.Y[m], cyl.Z[m]]) + p_cyl[9:]
    poses = np.stack([W.IDENTITY_POSE, p_cyl, W.pose12(np.eye(3), centre)])[None]
    fields = np.random.default_rng(5).standard_normal((4, bg.nodes + cyl.nodes + ball.nodes))
    return W.Workload("seam", [bg, cyl, ball], nf=3, steps=1, poses=poses, fields=fields)


def test_buffer_wraps_two_tiles_across_a_thin_periodic_seam():
    w = seam_case()
    o = oracle.Oracle(w.grids, w.nf)
    r = o.step(w.poses[0], w.fields)
    # the case reaches j = 119 of the shell through the seam
    f = r["flags"][o.node_off[1]:o.node_off[2]].reshape(9, 121, 6)
    assert (f[4, 1, 2] & 3) == oracle.ST_HOLE
    # buffer nodes (radial layers 0-3; 4 and 5 are outer-boundary fringe) at j = 119
    assert ((f[:, 119, :4] & 3) == oracle.ST_FRINGE).sum() > 0
    assert ((f[:, 118, :4] & 3) == oracle.ST_FRINGE).sum() == 0
    _run_and_compare(w, [0])
    _run_and_compare(w, [0], options={"holecut_cull": 0})


def polar_turn_case():
    """A spherical shell (polar angle from its x axis with pole nodes at both
    ends, azimuth periodic, 16 azimuthal cells) in a Cartesian background,
    turned half a revolution about its own axis after step 0. The queries
    whose donors are the wedge cells round the axis then start their walk,
    from step 0's donor, in the cell across the axis from the one that holds
    them."""
    bg = W.cartesian_grid(48)
    sph = W.spherical_shell(8, 16, 9, 0.08, 0.3)
    sph.blank_kind = W.BLANK_SPHERE
    sph.blank_prm = (0.08,)
    sph.outer = (0, 2, 0, 0, 0, 0)
    c = (0.5, 0.5, 0.5)
    poses = np.stack([np.stack([W.IDENTITY_POSE, W.pose12(np.eye(3), c)]),
                      np.stack([W.IDENTITY_POSE, W.pose12(np.diag([1.0, -1.0, -1.0]), c)])])
    fields = np.random.default_rng(3).standard_normal((4, bg.nodes + sph.nodes))
    return W.Workload("polar", [bg, sph], nf=2, steps=2, poses=poses, fields=fields)


def test_fp64_walk_crosses_the_polar_axis():
    """Past a polar end the FP64 walk goes on in the cells across the axis of
    revolution: after the half turn all 56 queries with donors in the polar
    wedge cells are found by the walk (status FOUND), none by the
    brute-force scan of the control cell, which is where a walk that clamps
    at the pole sends them. Both steps match the oracle, through the five
    calls and through the native executor (bit for bit with the five
    calls)."""
    from paper_1910_09315_amd.assembly import Pipeline
    w = polar_turn_case()
    o = oracle.Oracle(w.grids, w.nf)
    a = _assembly(w)
    b = _assembly(w, capacity=a.capacity)
    pipe = Pipeline(b, a.capacity, native=True, stages=1)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    for t in range(2):
        a.step(poses[t])
        g = a.results()
        r = o.step(w.poses[t], w.fields)
        compare(o, w.poses[t], r, g, value_rtol=1e-12, s_tol=1e-12, qx_tol=1e-14)
        pipe.submit(t, poses[t])
        p = pipe.results(t)
        for k in ("flags", "q_node", "donor_grid", "donor_cell", "status", "s", "values"):
            assert np.array_equal(p[k], g[k], equal_nan=True), (t, k)
    pipe.join()
    nci, ncj, nck = 7, 16, 8
    polar = (r["donor_grid"] == 1) & np.isin(r["donor_cell"] // (nci * ncj), (0, nck - 1))
    assert polar.sum() == 56
    code = g["status"] & 3
    assert (code[polar] == 1).all(), np.bincount(code[polar], minlength=4)
    assert (a.ctx.status() & ~2) == 0


def test_fringe_compact_on_flags_of_another_hole_cut():
    """overset_fringe_compact finds the hole tiles from the flags it is given:
    two hole cuts (steps 0 and 2) into two buffers, then the fringe
    compaction of the first buffer, run after the second hole cut, still
    gives step 0's flags and query list, and the rest of that step matches
    the oracle."""
    from paper_1910_09315_amd import binding as B
    from paper_1910_09315_amd.assembly import StepBuffers
    w = W.c1_small(steps=3)
    o = oracle.Oracle(w.grids, w.nf)
    for precision, tol in (("fp64", dict(value_rtol=1e-12, s_tol=1e-12, qx_tol=1e-14)),
                           ("mixed", dict(value_rtol=1e-5, s_tol=1e-4, qx_tol=1e-6))):
        a = _assembly(w, precision)
        other = StepBuffers(a.dev, a.total, a.capacity, a.dtype)
        p0, p2 = a.as_poses(w.poses[0]), a.as_poses(w.poses[2])
        B.overset_holecut(a.ctx, p0, a.flags)
        B.overset_holecut(a.ctx, p2, other.flags)
        B.overset_fringe_compact(a.ctx, a.nf, a.flags, a.q_grid, a.q_node, a.capacity, a.d_count)
        a.back(p0, a.buf)
        g = a.results()
        r = o.step(w.poses[0], w.fields)
        st = compare(o, w.poses[0], r, g, **tol)
        print("fringe on step-0 flags after the step-2 hole cut", precision, st, flush=True)
        # and the other buffer's own fringe pass gives step 2
        B.overset_fringe_compact(a.ctx, a.nf, other.flags, other.q_grid, other.q_node, a.capacity, other.d_count)
        a.back(p2, other)
        compare(o, w.poses[2], o.step(w.poses[2], w.fields), a.results(other), **tol)
        assert (a.ctx.status() & ~2) == 0


@pytest.mark.parametrize("alone", [True, False])
def test_executor_stage_timing_counts_from_the_next_step(alone):
    """ov_pipe_set_timing times the next submitted step and every `every`-th
    one after it, whatever the executor's step count when it is called."""
    from paper_1910_09315_amd.assembly import Pipeline
    w = W.c1_small(steps=12)
    a = _assembly(w, "fp64")
    pipe = Pipeline(a, a.capacity, native=True, stages=3, max_timed=16)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    for t in range(5):
        pipe.submit(t, poses[t])
    pipe.native.stage_times(0)
    pipe.native.set_timing(3, 2, alone=alone)
    for t in range(5, 12):
        pipe.submit(t, poses[t])
    pipe.join()
    torch.cuda.synchronize()
    pipe.native.set_timing(0)
    ms = pipe.native.stage_times(16)
    assert len(ms) == 3 and all(x > 0 for x in ms)  # steps 5, 8 and 11
    pipe.close()

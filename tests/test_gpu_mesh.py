"""GPU parity of the hole cut against closed surface triangulations (ray
parity, Sec. 2.2.2): the school with triangulated blank ellipsoids through
the whole step, against the CPU oracle on the same seeded inputs (flags,
query list, orphans and gated donors bit-exact). Needs an MI355X."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from parity import compare

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(value_rtol=1e-12, s_tol=1e-12, qx_tol=1e-14),
       "mixed": dict(value_rtol=1e-5, s_tol=1e-4, qx_tol=1e-6)}


def _assembly(w, precision, options=None, capacity=None):
    from paper_1910_09315_amd.assembly import Assembly
    a = Assembly(w.grids, w.nf, fields=w.fields, precision=precision, options=options)
    a.allocate(capacity or 2 * a.count_queries(w.poses[0]) + 1024)
    return a


@pytest.mark.parametrize("precision,options", [("fp64", None), ("mixed", None), ("fp64", {"holecut_cull": 0}),
                                               ("mixed", {"holecut_npl": 4}), ("mixed", {"holecut_list": 1}),
                                               ("fp64", {"holecut_list": 1})])
def test_triangulated_school_matches_oracle_every_step(precision, options):
    w = W.c3_mesh_small(steps=4)
    o = oracle.Oracle(w.grids, w.nf)
    a = _assembly(w, precision, options)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    holes = 0
    for t in range(w.steps):
        a.step(poses[t])
        g = a.results()
        r = o.step(w.poses[t], w.fields)
        st = compare(o, w.poses[t], r, g, **TOL[precision])
        holes += int(np.count_nonzero((r["flags"] & 3) == oracle.ST_HOLE))
        print(w.name, precision, options, t, st, flush=True)
    assert holes > 1000
    assert (a.ctx.status() & ~2) == 0


def test_triangulated_school_pipeline_matches_sequential():
    from paper_1910_09315_amd.assembly import Pipeline
    w = W.c3_mesh_small(steps=5)
    a = _assembly(w, "mixed")
    b = _assembly(w, "mixed", options={"field_layout": 1}, capacity=a.capacity)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    seq = []
    for t in range(w.steps):
        a.step(poses[t])
        seq.append(a.results())
    pipe = Pipeline(b, a.capacity, native=True, stages=3)
    for t in range(w.steps):
        pipe.submit(t, poses[t])
        if t >= 1:
            r = pipe.results(t - 1)
            for k in ("flags", "q_node", "donor_grid", "donor_cell", "status", "s"):
                assert np.array_equal(r[k], seq[t - 1][k], equal_nan=True), (t - 1, k)
            assert np.allclose(r["values"], seq[t - 1]["values"], rtol=0, atol=0, equal_nan=True)
    pipe.join()
    torch.cuda.synchronize()


def test_full_size_triangulated_school_sampled_steps():
    """C3M (384x256x256 background, 8 fish with 9,024-triangle blank
    surfaces) through the three-stream executor, checked at two steps."""
    from paper_1910_09315_amd.assembly import Assembly, Pipeline
    w = W.c3_mesh(steps=60)
    o = oracle.Oracle(w.grids, w.nf)
    a = Assembly(w.grids, w.nf, fields=w.fields, precision="mixed", options={"field_layout": 1})
    cap = 2 * a.count_queries(w.poses[0]) + 4096
    a.allocate(cap)
    pipe = Pipeline(a, cap, native=True, stages=3)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    for t in range(w.steps):
        pipe.submit(t, poses[t])
        if t in (0, 59):
            r = o.step(w.poses[t], w.fields)
            st = compare(o, w.poses[t], r, pipe.results(t), **TOL["mixed"])
            print("C3M", t, st, flush=True)
    pipe.join()
    torch.cuda.synchronize()
    assert (a.ctx.status() & ~2) == 0


def test_mesh_arguments_rejected():
    import paper_1910_09315_amd.binding as B
    w = W.c3_mesh_small(steps=1)
    ctx = B.Context(0, "fp64")
    g = w.grids[0]
    X, Y, Z = (torch.as_tensor(np.ascontiguousarray(getattr(g, k), dtype=np.float64)).cuda() for k in "XYZ")
    gid = ctx.grid_add(g.dims, g.periodic, X, Y, Z)
    tri = w.grids[1].blank_mesh
    with pytest.raises(B.OversetError):
        ctx.set_blank_mesh(gid + 1, tri)  # no such grid
    with pytest.raises(B.OversetError):
        ctx.set_blank_mesh(gid, tri[:3])  # not a closed surface
    bad = tri.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(B.OversetError):
        ctx.set_blank_mesh(gid, bad)
    ctx.set_blank_mesh(gid, tri)
    ctx.finalize()
    with pytest.raises(B.OversetError):
        ctx.set_blank_mesh(gid, tri)  # after finalize

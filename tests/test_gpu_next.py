"""GPU parity of the velocity-frame transformation (Sec. 2.3) and of the
interpolation matrix with its application (Sec. 2.2.6 second option,
Alg. 4): the HIP library through its C ABI against the CPU oracle on the
same seeded inputs, compared on the queries whose donors the oracle fixes
(margin >= 1e-3), with the rest checked for validity. Needs an MI355X."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from parity import compare

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(value_rtol=1e-12, s_tol=1e-12, qx_tol=1e-14),
       "mixed": dict(value_rtol=1e-5, s_tol=1e-4, qx_tol=1e-6)}
# weight tolerance: a weight is a product of three factors each within s_tol
W_TOL = {"fp64": 4e-12, "mixed": 4e-4}


def _assembly(w, precision, options=None, capacity=None):
    from paper_1910_09315_amd.assembly import Assembly
    a = Assembly(w.grids, w.nf, fields=w.fields, precision=precision, options=options)
    a.allocate(capacity or 2 * a.count_queries(w.poses[0]) + 1024)
    return a


def _workload(name):
    return {"c1_small": lambda: W.c1_small(steps=4), "c3_small": lambda: W.c3_small(steps=3),
            "c0": W.c0}[name]()


@pytest.mark.parametrize("name,precision", [("c1_small", "fp64"), ("c1_small", "mixed"), ("c3_small", "fp64"),
                                            ("c3_small", "mixed")])
def test_frame_velocity_matches_oracle(name, precision):
    """overset_interp followed by overset_frame_velocity against the
    oracle's interpolation turned into each receiver's frame."""
    w = _workload(name)
    o = oracle.Oracle(w.grids, w.nf)
    a = _assembly(w, precision, options={"frame_velocity": 1})
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    turn = 0.0
    for t in range(w.steps):
        a.step(poses[t])
        g = a.results()
        r = o.step(w.poses[t], w.fields)
        turned = oracle.frame_velocity(w.poses[t], r["q_grid"], r["donor_grid"], r["values"])
        ok = r["donor_grid"] >= 0
        turn = max(turn, np.abs(turned[0:3, ok] - r["values"][0:3, ok]).max())
        st = compare(o, w.poses[t], dict(r, values=turned), g, **TOL[precision])
        print(name, precision, t, st, flush=True)
    # the run really turns velocities: some receivers' frames differ from their donors'
    assert turn > 1e-2
    assert (a.ctx.status() & ~2) == 0


@pytest.mark.parametrize("stages,precision", [(1, "fp64"), (3, "mixed"), (2, "fp64")])
def test_frame_velocity_in_the_back_kernel_matches_the_separate_call(stages, precision):
    """The executors' one-kernel back half with the rotation inside equals
    the five calls followed by overset_frame_velocity, bitwise."""
    from paper_1910_09315_amd.assembly import Pipeline
    w = W.c1_small(steps=6)
    a = _assembly(w, precision, options={"frame_velocity": 1})
    b = _assembly(w, precision, options={"frame_velocity": 1}, capacity=a.capacity)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    seq = []
    for t in range(w.steps):
        a.step(poses[t])
        seq.append(a.results())
    pipe = Pipeline(b, a.capacity, native=True, stages=stages)
    lag = 0 if stages == 1 else 1
    for t in range(w.steps):
        pipe.submit(t, poses[t])
        if t >= lag:
            r = pipe.results(t - lag)
            for k in ("donor_grid", "donor_cell", "s", "values"):
                assert np.array_equal(r[k], seq[t - lag][k], equal_nan=True), (t - lag, k)
    pipe.join()
    torch.cuda.synchronize()


def _matrix_case(w, t, precision):
    o = oracle.Oracle(w.grids, w.nf)
    a = _assembly(w, precision)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    for k in range(t + 1):
        a.step(poses[k])
    cols, vals = a.interp_matrix()
    g = a.results()
    r = o.step(w.poses[t], w.fields)
    compare(o, w.poses[t], r, g, **TOL[precision])
    n = g["count"]
    return o, a, r, g, cols, vals, n


@pytest.mark.parametrize("name,precision", [("c0", "fp64"), ("c1_small", "fp64"), ("c1_small", "mixed"),
                                            ("c3_small", "mixed")])
def test_interp_matrix_matches_oracle(name, precision):
    """Columns bit-exact and weights within tolerance on every query whose
    donor the oracle fixes; rows of other donors index their own donor grid
    and sum to one; orphan rows are empty."""
    w = _workload(name)
    o, a, r, g, cols, vals, n = _matrix_case(w, w.steps - 1, precision)
    gc = cols[:n].cpu().numpy()
    gv = vals[:n].double().cpu().numpy()
    rc, rv = oracle.interp_matrix(o, r["donor_grid"], r["donor_cell"], r["s"])
    orphan = r["donor_grid"] < 0
    assert np.all(gc[orphan] == -1) and np.all(gv[orphan] == 0.0)
    fixed = ~orphan & (r["margin"] >= 1e-3)
    assert fixed.sum() > 0
    assert np.array_equal(gc[fixed], rc[fixed])
    assert np.abs(gv[fixed] - rv[fixed]).max() <= W_TOL[precision]
    live = ~orphan
    lo = o.node_off[g["donor_grid"][live]][:, None]
    hi = o.node_off[g["donor_grid"][live] + 1][:, None]
    assert np.all((gc[live] >= lo) & (gc[live] < hi))
    assert np.abs(gv[live].sum(axis=1) - 1.0).max() <= (1e-14 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("name,precision,nrhs", [("c1_small", "fp64", 1), ("c1_small", "fp64", 5),
                                                 ("c3_small", "mixed", 4)])
def test_interp_apply_matches_oracle(name, precision, nrhs):
    """y = M x on seeded vectors against the oracle's product of its own
    matrix, on the queries whose donor it fixes (normwise per vector), and
    M applied to the flow fields equals the interpolation."""
    w = _workload(name)
    o, a, r, g, cols, vals, n = _matrix_case(w, w.steps - 1, precision)
    rng = np.random.default_rng(1234 + nrhs)
    x = rng.standard_normal((nrhs, a.total))
    xd = torch.as_tensor(x).to(a.dtype).cuda().contiguous()
    y = a.interp_apply(cols, vals, xd)
    torch.cuda.synchronize()
    gy = y[:, :n].double().cpu().numpy()
    rc, rv = oracle.interp_matrix(o, r["donor_grid"], r["donor_cell"], r["s"])
    ry = oracle.matrix_apply(rc, rv, x)
    fixed = (r["donor_grid"] >= 0) & (r["margin"] >= 1e-3)
    tol = 1e-12 if precision == "fp64" else 1e-5
    for k in range(nrhs):
        assert np.abs(gy[k, fixed] - ry[k, fixed]).max() <= tol * np.abs(ry[k, fixed]).max()
    assert np.all(gy[:, r["donor_grid"] < 0] == 0.0)
    # the matrix applied to the fields (blocks u, v, w, p) is the interpolation
    f = torch.as_tensor(np.asarray(w.fields).reshape(4, a.total)).to(a.dtype).cuda().contiguous()
    yf = a.interp_apply(cols, vals, f)[:, :n].double().cpu().numpy()
    live = g["donor_grid"] >= 0
    scale = np.abs(g["values"][:, live]).max(axis=1, keepdims=True)
    assert np.all(np.abs(yf[:, live] - g["values"][:, live]) <= (1e-13 if precision == "fp64" else 1e-5) * scale)


@pytest.mark.parametrize("precision,nrhs", [("fp64", 4), ("mixed", 4), ("fp64", 3), ("mixed", 1)])
def test_interp_apply_interleaved_equals_blocks(precision, nrhs):
    """Vectors interleaved per node (one gather per corner with 4 vectors)
    give the blocks layout's results bitwise."""
    w = W.c3_small(steps=2)
    a = _assembly(w, precision)
    poses = torch.as_tensor(w.poses.reshape(w.steps, -1)).cuda()
    for k in range(w.steps):
        a.step(poses[k])
    cols, vals = a.interp_matrix()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(99)
    x = torch.randn((nrhs, a.total), generator=gen, dtype=torch.float64, device="cuda").to(a.dtype).contiguous()
    yb = a.interp_apply(cols, vals, x)
    yi = a.interp_apply(cols, vals, x.t().contiguous(), layout=1)
    torch.cuda.synchronize()
    n = int(a.d_count.item())
    assert n > 10000
    assert torch.equal(yi[:n].t(), yb[:, :n])


def test_matrix_calls_with_no_rows_and_bad_arguments():
    """Zero rows leave the outputs untouched; bad arguments are errors
    before any launch."""
    import paper_1910_09315_amd.binding as B
    w = W.c1_small(steps=1)
    a = _assembly(w, "fp64")
    a.d_count.zero_()
    cols = torch.full((a.capacity, 8), 77, dtype=torch.int32, device="cuda")
    vals = torch.full((a.capacity, 8), 5.0, dtype=torch.float64, device="cuda")
    B.overset_interp_matrix(a.ctx, a.donor_grid, a.donor_cell, a.s, a.d_count, a.capacity, cols, vals)
    y = torch.full((2, a.capacity), 3.0, dtype=torch.float64, device="cuda")
    x = torch.zeros((2, a.total), dtype=torch.float64, device="cuda")
    B.overset_interp_apply(a.ctx, cols, vals, a.d_count, a.capacity, x, 2, y)
    torch.cuda.synchronize()
    assert bool((cols == 77).all()) and bool((vals == 5.0).all()) and bool((y == 3.0).all())
    with pytest.raises(B.OversetError):
        B.overset_interp_apply(a.ctx, cols, vals, a.d_count, a.capacity, x, -1, y)
    with pytest.raises(B.OversetError):
        B.overset_interp_apply(a.ctx, cols, vals, a.d_count, a.capacity, x, 2, y, layout=2)
    with pytest.raises(B.OversetError):  # interleaved 4-vector gathers need 32-byte aligned fp64 values
        B.overset_interp_apply(a.ctx, cols, vals, a.d_count, a.capacity, x.reshape(-1)[1:], 4, y, layout=1)
    with pytest.raises(B.OversetError):
        B.overset_interp_matrix(a.ctx, a.donor_grid, a.donor_cell, None, a.d_count, a.capacity, cols, vals)
    with pytest.raises(B.OversetError):
        B.overset_frame_velocity(a.ctx, None, a.q_grid, a.donor_grid, a.d_count, a.capacity, a.out)

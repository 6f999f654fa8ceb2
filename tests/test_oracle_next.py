"""Pins of the oracle's velocity-frame transformation (Sec. 2.3) and of the
interpolation matrix and its application (Sec. 2.2.6 second option, Alg. 4)
against facts the paper and the mathematics fix: a uniform inertial
velocity seen from every frame, the partition of unity of the weights, and
the trilinear map of the donor's own coordinates reproducing the query's
position in the donor's frame. CPU only."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _rot(pose):
    return np.asarray(pose[:9], dtype=np.float64).reshape(3, 3)


def _uniform_inertial_velocity_fields(w, t, U):
    """Each grid's fields hold the components of one inertial velocity U in
    that grid's frame (R_g^T U at every node), and p = 7."""
    F = np.zeros((4, w.total_nodes))
    off = w.node_offsets
    for g in range(w.ngrids):
        F[0:3, off[g]:off[g + 1]] = (_rot(w.poses[t, g]).T @ U)[:, None]
    F[3] = 7.0
    return F


@pytest.mark.parametrize("make", [lambda: W.c1_small(steps=3), lambda: W.c3_small(steps=2)])
def test_uniform_inertial_velocity_arrives_in_the_receivers_frame(make):
    w = make()
    t = w.steps - 1
    U = np.array([0.3, -1.2, 0.75])
    o = oracle.Oracle(w.grids, w.nf)
    r = o.step(w.poses[t], _uniform_inertial_velocity_fields(w, t, U))
    ok = r["donor_grid"] >= 0
    assert ok.sum() > 0
    # the donors are in other, differently rotated frames
    assert np.any(r["donor_grid"][ok] != r["q_grid"][ok])
    v = oracle.frame_velocity(w.poses[t], r["q_grid"], r["donor_grid"], r["values"])
    want = np.stack([_rot(w.poses[t, a]).T @ U for a in r["q_grid"][ok]], axis=1)
    assert np.abs(v[0:3, ok] - want).max() <= 1e-12
    # without the transformation the receivers would see the donors' components
    rotated = [a for a, b in zip(r["q_grid"][ok], r["donor_grid"][ok])
               if not np.allclose(_rot(w.poses[t, a]), _rot(w.poses[t, b]))]
    assert rotated and np.abs(r["values"][0:3, ok] - want).max() > 1e-3
    assert np.array_equal(v[3], r["values"][3])  # pressure is a scalar
    assert np.all(np.isnan(v[:, ~ok]) == np.isnan(r["values"][:, ~ok]))


def _step(w, t):
    o = oracle.Oracle(w.grids, w.nf)
    return o, o.step(w.poses[t], w.fields)


def test_matrix_rows_sum_to_one_and_index_the_donor_grid():
    w = W.c1_small(steps=2)
    o, r = _step(w, 1)
    cols, vals = oracle.interp_matrix(o, r["donor_grid"], r["donor_cell"], r["s"])
    ok = r["donor_grid"] >= 0
    assert np.abs(vals[ok].sum(axis=1) - 1.0).max() <= 1e-14
    assert np.all(vals[ok] >= -1e-15)
    lo = o.node_off[r["donor_grid"][ok]][:, None]
    hi = o.node_off[r["donor_grid"][ok] + 1][:, None]
    assert np.all((cols[ok] >= lo) & (cols[ok] < hi))


def test_matrix_reproduces_query_positions_in_the_donor_frame():
    """Applied to the packed body-frame coordinates, row q gives the
    trilinear map of its donor cell at s: the query's own position in the
    donor's frame, computed here from its grid's pose."""
    w = W.c1_small(steps=2)
    t = 1
    o, r = _step(w, t)
    cols, vals = oracle.interp_matrix(o, r["donor_grid"], r["donor_cell"], r["s"])
    XYZ = np.stack([np.concatenate([np.asarray(getattr(g, c), dtype=np.float64).ravel() for g in w.grids])
                    for c in "XYZ"])
    got = oracle.matrix_apply(cols, vals, XYZ)
    ok = np.flatnonzero(r["donor_grid"] >= 0)
    for q in ok:
        A, m, B = r["q_grid"][q], r["q_node"][q], r["donor_grid"][q]
        g = w.grids[A]
        X = np.array([g.X.ravel()[m], g.Y.ravel()[m], g.Z.ravel()[m]])
        pa, pb = w.poses[t, A], w.poses[t, B]
        x = _rot(pa) @ X + pa[9:]
        xi = _rot(pb).T @ (x - pb[9:])
        assert np.abs(got[:, q] - xi).max() <= 1e-11, (q, got[:, q], xi)


def test_matrix_apply_equals_interpolation_and_orphan_rows_are_empty():
    w = W.c0()
    o, r = _step(w, 0)
    cols, vals = oracle.interp_matrix(o, r["donor_grid"], r["donor_cell"], r["s"])
    orphan = r["donor_grid"] < 0
    assert orphan.sum() == 144
    assert np.all(cols[orphan] == -1) and np.all(vals[orphan] == 0.0)
    y = oracle.matrix_apply(cols, vals, w.fields)
    ok = ~orphan
    assert np.abs(y[:, ok] - r["values"][:, ok]).max() <= 1e-14 * max(1.0, np.abs(r["values"][:, ok]).max())
    assert np.all(y[:, orphan] == 0.0)

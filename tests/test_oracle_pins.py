"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not by the oracle's own code: hand-derived counts, closed-form inverse maps of
box, cylindrical and spherical cells, lattice-point counts, brute force on
tiny grids, interpolation identities and error bounds. CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle_helpers import cell_index, interp_points, points_grid, search_points

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ------------------------------------------------------------------ P10: C0 counts
def test_c0_counts_match_hand_derivation():
    g = json.load(open(os.path.join(GOLDEN, "c0_counts.json")))
    w = W.c0()
    o = oracle.Oracle(w.grids, w.nf)
    r = o.step(w.poses[0], w.fields)
    off = o.node_off
    holes = (r["holecut_flags"] & 3) == oracle.ST_HOLE
    assert holes.sum() == g["holes"]
    hi = np.flatnonzero(holes)
    i, j, k = hi % 32, (hi // 32) % 32, hi // 1024
    assert sorted(set(zip(i.tolist(), j.tolist()))) == [tuple(x) for x in g["hole_columns_ij"]]
    assert (k.min(), k.max()) == tuple(g["hole_k_range"])
    f = r["flags"]
    assert ((f[: off[1]] & 3) == oracle.ST_FRINGE).sum() == g["background_fringe"]
    assert ((f[off[1]:] & 3) == oracle.ST_FRINGE).sum() == g["overset_fringe"]
    assert len(r["q_grid"]) == g["queries"]
    orph = r["donor_grid"] < 0
    assert orph.sum() == g["orphans"]
    # orphans are exactly the background buffer nodes beyond the shell's axial extent
    on = r["q_node"][orph]
    assert np.all(r["q_grid"][orph] == 0)
    assert sorted(set((on // 1024).tolist())) == g["orphan_k_layers"]
    # every background buffer node is caused by the overset (grid 1), donors come from it
    bgq = (r["q_grid"] == 0) & ~orph
    assert np.all(r["donor_grid"][bgq] == 1)
    assert np.all(r["donor_grid"][r["q_grid"] == 1] == 0)


# ------------------------------------------------------------------ P3: affine closed form
def test_box_cells_closed_form():
    rng = np.random.default_rng(3)
    dims, h, x0 = (7, 5, 6), np.array([0.3, 0.2, 0.45]), np.array([-1.0, 0.5, 2.0])
    g = W.cartesian_grid(dims, lo=x0, hi=x0 + h * (np.array(dims) - 1))
    R = W.rodrigues(rng.normal(size=3), 0.7)
    c = np.array([0.3, -0.2, 1.1])
    n = 400
    idx = np.stack([rng.integers(0, d - 1, n) for d in dims], 1)
    s = rng.uniform(1e-3, 1 - 1e-3, (n, 3))
    body = x0 + (idx + s) * h
    world = body @ R.T + c
    d = search_points(g, world, donor_pose=W.pose12(R, c))
    want = cell_index(dims, 0, idx[:, 0], idx[:, 1], idx[:, 2])
    assert np.array_equal(d["donor_cell"], want)
    assert np.abs(d["s"] - s).max() < 1e-12


def test_box_point_outside_is_orphan():
    g = W.cartesian_grid(4)
    d = search_points(g, [[1.5, 0.5, 0.5], [0.5, -0.01, 0.5], [0.5, 0.5, 0.5]])
    assert d["donor_grid"].tolist() == [-1, -1, 0]


# ------------------------------------------------------------------ P4: cylindrical closed form
def _cyl_inverse(q, r, th, z):
    """Closed-form natural coordinates in a cylindrical shell whose cells are
    bilinear in (r, angle) and affine in z: constant-angle-coordinate lines are
    rays through the axis, so t solves A x q + t ((D - A) x q) = 0 in 2D and the
    radius along that ray is |q| / |(1 - t) A + t D|."""
    phi = math.atan2(q[1], q[0]) % (2 * math.pi)
    nth = len(th)
    j = int(phi // (2 * math.pi / nth)) % nth
    A = np.array([math.cos(th[j]), math.sin(th[j])])
    D = np.array([math.cos(th[(j + 1) % nth]), math.sin(th[(j + 1) % nth])])
    cross = lambda a, b: a[0] * b[1] - a[1] * b[0]
    t = cross(A, q[:2]) / cross(A - D, q[:2])
    rho = math.hypot(q[0], q[1]) / np.linalg.norm((1 - t) * A + t * D)
    i = int(np.searchsorted(r, rho, side="right") - 1)
    if i < 0 or i >= len(r) - 1:
        return None, None
    sr = (rho - r[i]) / (r[i + 1] - r[i])
    k = int(np.searchsorted(z, q[2], side="right") - 1)
    sz = (q[2] - z[k]) / (z[k + 1] - z[k])
    return (i, j, k), np.array([sr, t, sz])


def test_cylindrical_cells_closed_form():
    rng = np.random.default_rng(4)
    w = W.c0()
    cyl = w.grids[1]
    pose = w.poses[0, 1]
    R, c = pose[:9].reshape(3, 3), pose[9:]
    r = np.linspace(0.05, 0.2, 16)
    th = 2 * math.pi * np.arange(16) / 16
    z = np.linspace(0.3, 0.7, 16)
    pts, cells, ss = [], [], []
    while len(pts) < 300:
        rho = rng.uniform(0.05, 0.2)
        ang = rng.uniform(0, 2 * math.pi)
        q = np.array([rho * math.cos(ang), rho * math.sin(ang), rng.uniform(0.3, 0.7)])
        cell, s = _cyl_inverse(q, r, th, z)
        if cell is None or min(s.min(), (1 - s).min()) < 1e-3:
            continue
        pts.append(R @ q + c)
        cells.append(cell_index(cyl.dims, cyl.periodic, *cell))
        ss.append(s)
    d = search_points(cyl, np.array(pts), donor_pose=pose)
    assert np.array_equal(d["donor_cell"], np.array(cells))
    assert np.abs(d["s"] - np.array(ss)).max() < 1e-11


# ------------------------------------------------------------------ P5: spherical closed form
def test_spherical_cells_closed_form():
    """Points built in factored form p = rho(s_r) * B(t, u), B the bilinear
    blend of the cell's four unit-sphere corner directions: that is the
    trilinear map of a spherical-shell cell, whose radial lines pass through
    the centre. Includes the degenerate polar cells."""
    rng = np.random.default_rng(5)
    nr, nphi, nth, r0, r1 = 5, 12, 7, 0.3, 0.9
    g = W.spherical_shell(nr, nphi, nth, r0, r1)
    rr = np.linspace(r0, r1, nr)
    phi = 2 * math.pi * np.arange(nphi) / nphi
    th = math.pi * np.arange(nth) / (nth - 1)

    def unit(j, k):
        st = 0.0 if k in (0, nth - 1) else math.sin(th[k])
        ct = 1.0 if k == 0 else (-1.0 if k == nth - 1 else math.cos(th[k]))
        return np.array([ct, st * math.cos(phi[j % nphi]), st * math.sin(phi[j % nphi])])

    pose = W.pose12(W.rodrigues((1, 2, 3), 0.4), (0.1, 0.2, 0.3))
    R, c = pose[:9].reshape(3, 3), pose[9:]
    pts, cells, ss = [], [], []
    for _ in range(300):
        i, j, k = rng.integers(0, nr - 1), rng.integers(0, nphi), rng.integers(0, nth - 1)
        s = rng.uniform(1e-3, 1 - 1e-3, 3)
        B = ((1 - s[1]) * (1 - s[2]) * unit(j, k) + s[1] * (1 - s[2]) * unit(j + 1, k)
             + (1 - s[1]) * s[2] * unit(j, k + 1) + s[1] * s[2] * unit(j + 1, k + 1))
        rho = (1 - s[0]) * rr[i] + s[0] * rr[i + 1]
        pts.append(R @ (rho * B) + c)
        cells.append(cell_index(g.dims, g.periodic, i, j, k))
        ss.append(s)
    d = search_points(g, np.array(pts), donor_pose=pose)
    assert np.array_equal(d["donor_cell"], np.array(cells))
    assert np.abs(d["s"] - np.array(ss)).max() < 1e-10


# ------------------------------------------------------------------ P1: control cells vs brute force
@pytest.mark.parametrize("seed,dims,periodic", [(1, (5, 4, 6), 0), (2, (8, 6, 5), 0), (3, (4, 7, 4), 0),
                                                (4, (6, 5, 5), 0), (5, (10, 10, 10), 0)])
def test_control_cells_equal_exhaustive(seed, dims, periodic):
    rng = np.random.default_rng(seed)
    g = W.perturbed_box_grid(rng, dims, h=0.1, amp=0.2, periodic=periodic)
    lo = np.array([g.X.min(), g.Y.min(), g.Z.min()]) - 0.05
    hi = np.array([g.X.max(), g.Y.max(), g.Z.max()]) + 0.05
    pts = rng.uniform(lo, hi, (600, 3))
    flags = np.zeros(g.nodes, np.uint8)
    flags[rng.integers(0, g.nodes, 3)] = oracle.ST_HOLE
    a = search_points(g, pts, donor_flags=flags)
    b = search_points(g, pts, donor_flags=flags, exhaustive=True)
    assert np.array_equal(a["donor_cell"], b["donor_cell"])
    assert np.array_equal(a["donor_grid"], b["donor_grid"])
    assert (a["donor_grid"] >= 0).sum() > 100


def test_control_cells_equal_exhaustive_periodic_ring():
    """A periodic direction: a ring of cells closing on itself (C0's shell)."""
    rng = np.random.default_rng(7)
    g = W.cylindrical_shell(4, 9, 4, 0.2, 0.5, 0.0, 0.3)
    pts = rng.uniform([-0.55, -0.55, -0.02], [0.55, 0.55, 0.32], (800, 3))
    a = search_points(g, pts)
    b = search_points(g, pts, exhaustive=True)
    assert np.array_equal(a["donor_cell"], b["donor_cell"])
    wrap = (a["donor_cell"] >= 0) & ((a["donor_cell"] // 3) % 9 == 8)
    assert wrap.sum() > 10   # the wrap cell (j = 8 -> 0) is found


# ------------------------------------------------------------------ P2: generated in-cell queries
def _forward(P, s):
    """x(s) for corners P[8,3] (corner c = c0 + 2 c1 + 4 c2)."""
    x = np.zeros(3)
    for c in range(8):
        b = [(c >> d) & 1 for d in range(3)]
        wgt = np.prod([s[d] if b[d] else 1 - s[d] for d in range(3)])
        x += wgt * P[c]
    return x


def test_generated_in_cell_queries_recover_cell_and_s():
    rng = np.random.default_rng(8)
    g = W.perturbed_box_grid(rng, (6, 7, 5), h=1.0, amp=0.2)
    ni, nj, nk = g.dims
    pts, cells, ss = [], [], []
    for _ in range(300):
        ci, cj, ck = rng.integers(0, ni - 1), rng.integers(0, nj - 1), rng.integers(0, nk - 1)
        P = np.array([[g.X[m], g.Y[m], g.Z[m]] for m in
                      [(ci + (c & 1)) + ni * ((cj + ((c >> 1) & 1)) + nj * (ck + (c >> 2))) for c in range(8)]])
        s = rng.uniform(1e-3, 1 - 1e-3, 3)
        pts.append(_forward(P, s))
        cells.append(cell_index(g.dims, 0, ci, cj, ck))
        ss.append(s)
    d = search_points(g, np.array(pts))
    assert np.array_equal(d["donor_cell"], np.array(cells))
    assert np.abs(d["s"] - np.array(ss)).max() < 1e-12


# ------------------------------------------------------------------ P6: linear reproduction
def test_linear_field_reproduced_exactly():
    rng = np.random.default_rng(9)
    g = W.perturbed_box_grid(rng, (6, 6, 6), h=0.2, amp=0.2)
    lin = lambda x, y, z: 1 + 2 * x - 3 * y + 0.5 * z
    F = np.stack([lin(g.X, g.Y, g.Z), -lin(g.X, g.Y, g.Z)])
    pts = rng.uniform([0.2, 0.2, 0.2], [0.8, 0.8, 0.8], (500, 3))
    d, vals = interp_points(g, pts, F)
    ok = d["donor_grid"] >= 0
    assert ok.sum() > 400
    want = lin(pts[:, 0], pts[:, 1], pts[:, 2])
    assert np.abs(vals[0][ok] - want[ok]).max() <= 1e-12 * np.abs(want).max()
    assert np.abs(vals[1][ok] + want[ok]).max() <= 1e-12 * np.abs(want).max()


def test_trilinear_field_reproduced_on_box_cells():
    """On box cells a field trilinear in x, y, z (p = xyz) is reproduced."""
    rng = np.random.default_rng(10)
    g = W.cartesian_grid((5, 6, 7), lo=(0.1, 0.2, 0.3), hi=(0.9, 1.0, 1.2))
    F = (g.X * g.Y * g.Z)[None]
    pts = rng.uniform([0.1, 0.2, 0.3], [0.9, 1.0, 1.2], (300, 3))
    d, vals = interp_points(g, pts, F)
    want = pts[:, 0] * pts[:, 1] * pts[:, 2]
    assert np.abs(vals[0] - want).max() < 1e-12


# ------------------------------------------------------------------ P7: weight invariants
def test_weights_partition_of_unity_and_corners():
    rng = np.random.default_rng(11)
    for s in rng.uniform(0, 1, (200, 3)):
        w = oracle.weights(s)
        assert abs(w.sum() - 1.0) <= 1e-15
        assert w.min() >= 0
    for c in range(8):
        s = np.array([(c >> d) & 1 for d in range(3)], dtype=np.float64)
        w = oracle.weights(s)
        assert w[c] == 1.0 and np.count_nonzero(w) == 1


def test_corner_values_returned_exactly_and_in_i_order():
    """A point at node (i+1, j, k) of a box cell interpolates exactly that
    node's value: corner 1 is the +i neighbour, corner 2 the +j, corner 4 the +k."""
    g = W.cartesian_grid((4, 5, 6))
    vals = np.arange(g.nodes, dtype=np.float64) * 1.5 + 0.25
    ni, nj = 4, 5
    pts, want = [], []
    for (i, j, k) in [(1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2)]:
        pts.append([g.X[i + ni * (j + nj * k)], g.Y[i + ni * (j + nj * k)], g.Z[i + ni * (j + nj * k)]])
        want.append(vals[i + ni * (j + nj * k)])
    # nudge inside cell (1,1,1) so the cell is unique: s = (1e-13 or 1 - 1e-13)
    d, out = interp_points(g, np.array(pts) + np.array([1e-14, 1e-14, 1e-14]), vals[None])
    assert np.allclose(out[0], want, rtol=0, atol=1e-11)


# ------------------------------------------------------------------ P9: second order
def test_second_order_error_bound_and_rate():
    rng = np.random.default_rng(12)
    pts = rng.uniform(0.05, 0.95, (1500, 3))
    f = lambda x, y: np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y)
    errs = []
    for n in (17, 33, 65):
        g = W.cartesian_grid(n)
        h = 1.0 / (n - 1)
        d, vals = interp_points(g, pts, f(g.X, g.Y)[None])
        e = np.abs(vals[0] - f(pts[:, 0], pts[:, 1])).max()
        assert e <= (h * h / 8) * (2 * (2 * math.pi) ** 2) * (1 + 1e-9)
        errs.append(e)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, errs


# ------------------------------------------------------------------ P8: rigid invariance
def test_rigid_motion_of_everything_changes_nothing():
    w = W.c1_small(steps=2)
    o = oracle.Oracle(w.grids, w.nf)
    G = W.pose12(W.rodrigues((0.3, -1.0, 0.4), 1.1), (0.7, -0.4, 2.0))
    RG, cG = G[:9].reshape(3, 3), G[9:]
    p = w.poses[1]
    q = np.empty_like(p)
    for g in range(w.ngrids):
        R, c = p[g, :9].reshape(3, 3), p[g, 9:]
        q[g] = W.pose12(RG @ R, RG @ c + cG)
    a = o.step(p, w.fields)
    b = o.step(q, w.fields)
    assert np.array_equal(a["flags"], b["flags"])
    assert np.array_equal(a["q_node"], b["q_node"])
    gated = a["margin"] >= 1e-6
    assert np.array_equal(a["donor_cell"][gated], b["donor_cell"][gated])
    assert np.array_equal(a["donor_grid"] < 0, b["donor_grid"] < 0)
    assert np.nanmax(np.abs(a["s"][gated] - b["s"][gated])) < 1e-10


# ------------------------------------------------------------------ hole cut
def _holecut_points(pts, blank_kind, prm, pose):
    """Holes among world points `pts` (grid 0) cut by a blank region carried by
    a dummy grid 1 placed at `pose`."""
    pg = points_grid(pts)
    dummy = W.cartesian_grid(2, lo=(50, 50, 50), hi=(51, 51, 51))
    dummy.blank_kind, dummy.blank_prm = blank_kind, prm
    o = oracle.Oracle([pg, dummy], nf=0)
    flags, _ = o.holecut(np.stack([W.IDENTITY_POSE, pose]))
    return flags[: pg.nodes]


def test_sphere_blank_lattice_count():
    """Integer points strictly inside a sphere of radius^2 4.5 about a lattice
    point: norms^2 0, 1, 2, 3, 4 occur 1 + 6 + 12 + 8 + 6 = 33 times."""
    g = W.cartesian_grid(11, lo=(0, 0, 0), hi=(10, 10, 10))
    pts = np.stack([g.X, g.Y, g.Z], 1)
    fl = _holecut_points(pts, W.BLANK_SPHERE, (math.sqrt(4.5),), W.pose12(np.eye(3), (5, 5, 5)))
    assert ((fl & 3) == oracle.ST_HOLE).sum() == 33
    assert np.all(fl[(fl & 3) == oracle.ST_HOLE] >> 2 == 1)


def test_ellipsoid_blank_lattice_count():
    """Semi-axes (2.5, 1.5, 1.2): 5 points on the x axis, 3 x 2 with |y| = 1,
    3 x 2 with |z| = 1, none with |y| = |z| = 1: 17."""
    g = W.cartesian_grid(11, lo=(0, 0, 0), hi=(10, 10, 10))
    pts = np.stack([g.X, g.Y, g.Z], 1)
    fl = _holecut_points(pts, W.BLANK_ELLIPSOID, (2.5, 1.5, 1.2), W.pose12(np.eye(3), (4, 5, 6)))
    assert ((fl & 3) == oracle.ST_HOLE).sum() == 17


def test_blank_follows_rotation_direction():
    """Ellipsoid (2.5, 1.5, 1.5) rotated +30 deg about z: a point 2.4 along the
    +30 deg direction lies on its long axis (inside); one along -30 deg is
    (1.2, -2.08) in the body frame (outside)."""
    a = math.radians(30)
    pose = W.pose12(W.rot_z(a), (0, 0, 0))
    pts = [[2.4 * math.cos(a), 2.4 * math.sin(a), 0], [2.4 * math.cos(-a), 2.4 * math.sin(-a), 0]]
    fl = _holecut_points(pts, W.BLANK_ELLIPSOID, (2.5, 1.5, 1.5), pose)
    assert (fl & 3).tolist() == [oracle.ST_HOLE, oracle.ST_FIELD]


def test_cylinder_blank_axial_range_inclusive_radius_strict():
    pose = W.pose12(np.eye(3), (1, 1, 0))
    pts = [[1.0, 1.0, 0.3], [1.0, 1.0, 0.7], [1.0, 1.0, 0.2999], [1.5, 1.0, 0.5], [1.4999, 1, 0.5]]
    fl = _holecut_points(pts, W.BLANK_CYL, (0.5, 0.3, 0.7), pose)
    assert (fl & 3).tolist() == [1, 1, 0, 0, 1]


def test_hole_cause_is_lowest_blanking_grid():
    bg = W.cartesian_grid(9, lo=(0, 0, 0), hi=(8, 8, 8))
    g1 = W.cartesian_grid(2, lo=(50, 50, 50), hi=(51, 51, 51))
    g2 = W.cartesian_grid(2, lo=(60, 60, 60), hi=(61, 61, 61))
    g1.blank_kind, g1.blank_prm = W.BLANK_SPHERE, (1.5,)
    g2.blank_kind, g2.blank_prm = W.BLANK_SPHERE, (1.5,)
    o = oracle.Oracle([bg, g1, g2], nf=0)
    poses = np.stack([W.IDENTITY_POSE, W.pose12(np.eye(3), (4, 4, 4)), W.pose12(np.eye(3), (5, 4, 4))])
    fl, _ = o.holecut(poses)
    node = lambda i, j, k: i + 9 * (j + 9 * k)
    assert fl[node(4, 4, 4)] == (1 | (1 << 2))   # in both: lowest id wins
    assert fl[node(5, 4, 4)] == (1 | (1 << 2))
    assert fl[node(6, 4, 4)] == (1 | (2 << 2))   # only in grid 2's blank
    assert fl[node(3, 4, 4)] == (1 | (1 << 2))


# ------------------------------------------------------------------ fringe
def _fringe_single(dims, holes, nf, periodic=0, outer=(0,) * 6, cause=1):
    g = W.cartesian_grid(dims)
    g.periodic, g.outer = periodic, outer
    o = oracle.Oracle([g], nf)
    fl = np.zeros(g.nodes, np.uint8)
    ni, nj = g.dims[0], g.dims[1]
    for (i, j, k), c in zip(holes, cause if isinstance(cause, list) else [cause] * len(holes)):
        fl[i + ni * (j + nj * k)] = 1 | (c << 2)
    o.fringe(fl, nf)
    return fl


def test_buffer_of_single_hole_is_chebyshev_box():
    for nf, want in ((1, 26), (2, 124), (3, 342)):
        fl = _fringe_single((9, 9, 9), [(4, 4, 4)], nf)
        assert ((fl & 3) == oracle.ST_FRINGE).sum() == want
        assert np.all(fl[(fl & 3) == oracle.ST_FRINGE] >> 2 == 1)


def test_buffer_clipped_at_boundary_and_wrapped_when_periodic():
    fl = _fringe_single((9, 9, 9), [(0, 0, 0)], 2)
    assert ((fl & 3) == oracle.ST_FRINGE).sum() == 26           # 3^3 - 1
    fl = _fringe_single((9, 9, 9), [(0, 4, 4)], 1, periodic=1)
    fr = np.flatnonzero((fl & 3) == oracle.ST_FRINGE)
    assert ((fl & 3) == oracle.ST_FRINGE).sum() == 26
    assert set((fr % 9).tolist()) == {8, 0, 1}                  # i = -1 wraps to 8


def test_buffer_cause_is_min_and_boundary_layers():
    fl = _fringe_single((12, 5, 5), [(3, 2, 2), (6, 2, 2)], 2, cause=[5, 3])
    node = lambda i: i + 12 * (2 + 5 * 2)
    assert fl[node(1)] >> 2 == 5 and fl[node(4)] >> 2 == 3 and fl[node(8)] >> 2 == 3
    assert fl[node(3)] == 1 | (5 << 2)                          # holes untouched
    fl = _fringe_single((6, 7, 8), [], 2, outer=(0, 2, 0, 0, 0, 0))
    fr = (fl & 3) == oracle.ST_FRINGE
    assert fr.sum() == 2 * 7 * 8 and np.all(fl[fr] >> 2 == oracle.CAUSE_BOUNDARY)


def test_overset_fringe_count_is_layers_times_face():
    """Outer radial layers of a shell: nf x N_phi x N_theta queries (C1: 2 x 128 x 64)."""
    w = W.sphere_case("t", (24, 24, 24), (10, 16, 9), 0.1, 0.3, 1, seed=0)
    o = oracle.Oracle(w.grids, w.nf)
    r = o.step(w.poses[0], w.fields)
    ov = (r["flags"][o.node_off[1]:] & 3) == oracle.ST_FRINGE
    assert ov.sum() == 2 * 16 * 9


# ------------------------------------------------------------------ compaction
def test_compaction_is_ascending_and_complete():
    rng = np.random.default_rng(13)
    g0, g1 = W.cartesian_grid(5), W.cartesian_grid(4)
    o = oracle.Oracle([g0, g1], 0)
    fl = rng.integers(0, 3, o.total_nodes).astype(np.uint8)
    qg, qn = o.compact(fl)
    glob = o.node_off[qg] + qn
    assert np.all(np.diff(glob) > 0)
    assert np.array_equal(glob, np.flatnonzero((fl & 3) == 2))

"""Pins of the oracle's hole cut against a closed surface triangulation by
ray parity (Sec. 2.2.2: blank regions given by the body's surface
triangulation), against facts fixed independently of it: the half-space
description of a convex polyhedron (scipy's convex hull), exact projected
edge and vertex hits on an axis-aligned cube (each crossing counted once),
and the implicit ellipsoid a triangulation is inscribed in (agreement away
from the surface by more than the chord error). CPU only."""
import numpy as np
import pytest
from scipy.spatial import ConvexHull

import oracle
import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _hull_case(seed, npts=40):
    rng = np.random.default_rng(seed)
    pts = rng.standard_normal((npts, 3)) @ np.diag([1.0, 0.6, 0.8])
    hull = ConvexHull(pts)
    tri = pts[hull.simplices]
    return hull, tri


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_convex_polyhedron_matches_half_spaces(seed):
    hull, tri = _hull_case(seed)
    rng = np.random.default_rng(100 + seed)
    lo, hi = hull.points.min(0) - 0.3, hull.points.max(0) + 0.3
    p = rng.uniform(lo, hi, size=(20000, 3))
    # points whose ray passes exactly through a projected vertex or edge midpoint
    v = hull.points[hull.vertices]
    xs = rng.uniform(lo[0], hi[0], size=len(v))
    p_vert = np.column_stack([xs, v[:, 1], v[:, 2]])
    e = tri[:, [0, 1], :].mean(axis=1)
    p_edge = np.column_stack([rng.uniform(lo[0], hi[0], size=len(e)), e[:, 1], e[:, 2]])
    p = np.vstack([p, p_vert, p_edge])
    lhs = p @ hull.equations[:, :3].T + hull.equations[:, 3]
    inside = np.all(lhs < 0, axis=1)
    clear = np.all(np.abs(lhs) > 1e-9, axis=1)  # not on the surface
    got, gap = oracle.mesh_inside(tri, p)
    assert inside.sum() > 1000 and (~inside).sum() > 1000
    assert np.array_equal(got[clear], inside[clear])


def _cube():
    c = np.array([[x, y, z] for z in (-1, 1) for y in (-1, 1) for x in (-1, 1)], dtype=float)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    tri = []
    for a, b, cc, d in quads:
        tri += [(a, b, cc), (a, cc, d)]
    return c[np.array(tri)]


def test_cube_rays_through_projected_edges_and_vertices_count_once():
    """An axis-aligned cube: the x = +1 and x = -1 faces project onto the
    same square, split along a diagonal; the four faces parallel to x
    project edge-on and never count. Rays through the diagonal (a shared
    edge) and through the square's centre vertex must cross each face once."""
    tri = _cube()
    t = np.linspace(-0.75, 0.75, 7)
    pts, want = [], []
    for x, inside in ((-1.5, False), (-0.25, True), (0.5, True), (1.5, False)):
        for u in t:
            for y, z in ((u, u), (u, -u), (u, 0.3), (0.0, 0.0)):
                pts.append((x, y, z))
                want.append(inside)
    got, gap = oracle.mesh_inside(tri, np.array(pts))
    assert np.array_equal(got, np.array(want))


def _implicit_measure(w, t, B):
    """(x/a)^2 + (y/b)^2 + (z/c)^2 - 1 of every node of every grid in fish
    B's body frame (the implicit ellipsoid the triangulation is inscribed in)."""
    pose = w.poses[t, B]
    R, c = pose[:9].reshape(3, 3), pose[9:]
    a = np.asarray(w.grids[B].blank_prm[:3])
    out = []
    for g in w.grids:
        X = np.stack([np.asarray(getattr(g, k), dtype=np.float64).ravel() for k in "XYZ"])
        pg = w.poses[t, w.grids.index(g)]
        x = pg[:9].reshape(3, 3) @ X + pg[9:, None]
        xi = R.T @ (x - c[:, None])
        out.append(((xi / a[:, None]) ** 2).sum(0) - 1.0)
    return np.concatenate(out)


def test_triangulated_ellipsoids_agree_with_the_implicit_ones_away_from_the_surface():
    """C3M-small (320 triangles per fish) against the same school with the
    implicit ellipsoids: a node outside every implicit ellipsoid is no
    mesh hole (the triangulation is inscribed in a convex body), and a node
    deeper than the chord error (measure < -0.12; the faces stay within
    -0.04 of the surface) is a mesh hole."""
    wm = W.c3_mesh_small(steps=2)
    t = 1
    o = oracle.Oracle(wm.grids, wm.nf)
    fm, gap = o.holecut(wm.poses[t])
    assert gap > 1e-9
    hole = (fm & 3) == oracle.ST_HOLE
    fish = [B for B, g in enumerate(wm.grids) if g.blank_kind == W.BLANK_MESH]
    assert len(fish) == 8
    f = np.stack([_implicit_measure(wm, t, B) for B in fish])
    own = np.concatenate([np.full(g.nodes, i) for i, g in enumerate(wm.grids)])
    for k, B in enumerate(fish):
        f[k, own == B] = np.inf  # a grid does not cut itself
    outside_all = np.all(f >= 0, axis=0)
    deep = np.any(f < -0.12, axis=0)
    assert deep.sum() > 500
    assert not np.any(hole & outside_all)
    assert np.all(hole[deep])
    # the cause is the lowest fish whose mesh holds the node: where one fish is deep
    # and no lower one reaches, the cause is that fish
    first_deep = np.argmax(f < -0.12, axis=0)
    lower_clear = np.array([np.all(f[:first_deep[n], n] >= 0) for n in np.flatnonzero(deep)])
    sel = np.flatnonzero(deep)[lower_clear]
    assert np.array_equal((fm[sel] >> 2).astype(int), np.array(fish)[first_deep[sel]])

"""Pins of the oracle's donor selection (Sec. 2.4 item 1): which candidate
grid supplies the donor when a query point lies in several grids, and when a
containing cell is invalid because one of its corners is a hole. CPU only.

The grids are boxes of uniform cells placed by rigid poses, so every
containing cell and its natural coordinates follow in closed form from the
body-frame position (cell = floor((xi - lo) / h), s = the fractional part).
Each expected donor below is therefore fixed by that geometry and the rule
as stated: the query's cause grid first, then the background, then the other
grids in ascending id; a cell with a HOLE corner (in the donor grid's own
flags) is no donor, FRINGE corners are allowed; no valid containing cell in
any candidate grid makes an orphan.

Every pin is also run against variant builds of the oracle, each with one
plausible mistake planted in a copy of its C source (compiled on the CPU into
a temporary directory); each pin must fail on the variants named in its
docstring."""
import ctypes
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle_helpers import cell_index, search_points

HOLE = oracle.ST_HOLE
FRINGE = oracle.ST_FRINGE


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ------------------------------------------------------------------ geometry
def _box(n, half, name):
    return W.cartesian_grid((n, n, n), lo=(-half,) * 3, hi=(half,) * 3, name=name)


# background: 11^3 nodes on [0, 1]^3 (h = 0.1); two rotated overset boxes
# around the centre, both overlapping it and each other
GRIDS = [W.cartesian_grid((11, 11, 11)), _box(9, 0.2, "box1"), _box(7, 0.15, "box2")]
POSES = np.stack([W.IDENTITY_POSE,
                  W.pose12(W.rodrigues((1.0, 2.0, 3.0), 0.4), (0.48, 0.50, 0.52)),
                  W.pose12(W.rodrigues((-2.0, 1.0, 1.0), 0.9), (0.55, 0.47, 0.50))])
LO = [0.0, -0.2, -0.15]
H = [0.1, 0.05, 0.05]


def world(g, node):
    G = GRIDS[g]
    X = np.array([G.X[node], G.Y[node], G.Z[node]])
    R, c = POSES[g, :9].reshape(3, 3), POSES[g, 9:]
    return R @ X + c


def closed_form(g, x):
    """(cell, s, margin) of world point x in box grid g, or None if x lies
    outside it."""
    R, c = POSES[g, :9].reshape(3, 3), POSES[g, 9:]
    xi = R.T @ (x - c)
    u = (xi - LO[g]) / H[g]
    idx = np.floor(u).astype(int)
    n = GRIDS[g].dims[0]
    if np.any(idx < 0) or np.any(idx >= n - 1):
        return None
    s = u - idx
    return cell_index(GRIDS[g].dims, 0, *idx), s, float(min(s.min(), (1 - s).min()))


def corners(g, cell):
    n = GRIDS[g].dims[0]
    ci, cj, ck = cell % (n - 1), (cell // (n - 1)) % (n - 1), cell // (n - 1) ** 2
    return [(ci + (c & 1)) + n * ((cj + ((c >> 1) & 1)) + n * (ck + ((c >> 2) & 1))) for c in range(8)]


def nearest_nodes(g, target, k):
    G = GRIDS[g]
    P = np.stack([G.X, G.Y, G.Z], 1) @ POSES[g, :9].reshape(3, 3).T + POSES[g, 9:]
    return np.argsort(np.linalg.norm(P - target, axis=1))[:k].tolist()


OFF = np.concatenate([[0], np.cumsum([G.nodes for G in GRIDS])])


def search(queries, flags=None, extra=()):
    """Oracle donor search of queries [(grid, node, cause)]; flags default to
    FIELD everywhere; `extra` = [(grid, node, flag byte)] set afterwards."""
    o = oracle.Oracle(GRIDS, nf=0)
    f = np.zeros(o.total_nodes, np.uint8) if flags is None else flags.copy()
    for g, m, cause in queries:
        f[OFF[g] + m] = FRINGE | (cause << 2)
    for g, m, b in extra:
        f[OFF[g] + m] = b
    qg = np.array([q[0] for q in queries], np.int32)
    qn = np.array([q[1] for q in queries], np.int32)
    return o.donor_search(POSES, f, qg, qn)


def expect(d, i, g, x):
    """Query i must have its donor in grid g: the closed-form cell and s."""
    cf = closed_form(g, x)
    assert cf is not None, "test geometry: the point must lie in the expected grid"
    cell, s, m = cf
    assert m >= 1e-3, "test geometry: the point must lie clear of the expected cell's faces"
    assert d["donor_grid"][i] == g, f"query {i}: donor grid {d['donor_grid'][i]}, expected {g}"
    assert d["donor_cell"][i] == cell, f"query {i}: donor cell {d['donor_cell'][i]}, expected {cell}"
    assert np.abs(d["s"][i] - s).max() < 1e-12


def inside_all(x, grids):
    for g in grids:
        assert closed_form(g, x) is not None, f"test geometry: the point must lie in grid {g}"


# ------------------------------------------------------------------ pins
def check_priority():
    """Candidate order among three grids. Fails if the background is tried
    before the cause grid, if the cause is ignored (ascending ids first), or
    if an overset's outer-fringe point skips the background."""
    q = []
    # background buffer nodes cut by overset 2 / overset 1, inside both oversets
    b0 = 5 + 11 * (5 + 11 * 5)
    b1 = 5 + 11 * (4 + 11 * 5)
    q += [(0, b0, 2), (0, b1, 1)]
    # an overset-1 node in its outer fringe (cause 63) inside the background and overset 2
    n1 = nearest_nodes(1, POSES[2, 9:], 2)
    q += [(1, n1[0], oracle.CAUSE_BOUNDARY), (1, n1[1], 2)]
    # an overset-2 node cut by overset 1, inside the background and overset 1
    n2 = nearest_nodes(2, POSES[1, 9:], 1)
    q += [(2, n2[0], 1)]
    want = [2, 1, 0, 2, 1]
    competitors = [(1, 2), (1, 2), (0, 2), (0, 2), (0, 1)]
    d = search(q)
    for i, (g, m, _) in enumerate(q):
        x = world(g, m)
        inside_all(x, competitors[i])
        expect(d, i, want[i], x)


def check_hole_corner_in_donor_grid():
    """A containing cell with a HOLE corner in the donor grid's flags is no
    donor: the next candidate grid supplies it. Fails if the corner test
    reads the query grid's flags, or only recognises holes whose cause bits
    are zero."""
    m = nearest_nodes(1, POSES[2, 9:], 1)[0]
    x = world(1, m)
    inside_all(x, (0, 2))
    cell2 = closed_form(2, x)[0]
    hole = 1 | (1 << 2)  # a hole cut by grid 1
    d = search([(1, m, 2)], extra=[(2, corners(2, cell2)[7], hole)])
    expect(d, 0, 0, x)
    # every corner position invalidates the cell
    for c in range(8):
        d = search([(1, m, 2)], extra=[(2, corners(2, cell2)[c], hole)])
        assert d["donor_grid"][0] == 0, f"hole at corner {c} must invalidate the cell"


def check_fringe_corners_valid():
    """FRINGE corners (either cause) leave a cell valid, and HOLE flags at the
    same local indices of the query grid do not touch it. Fails if FRINGE
    corners are rejected, or if the query grid's flags are read."""
    m = nearest_nodes(1, POSES[2, 9:], 1)[0]
    x = world(1, m)
    cell2 = closed_form(2, x)[0]
    cn = corners(2, cell2)
    extra = [(2, cn[0], FRINGE | (oracle.CAUSE_BOUNDARY << 2)), (2, cn[5], FRINGE | (1 << 2))]
    # the query grid's nodes with the local indices of the donor cell's corners are holes
    extra += [(1, k, 1 | (2 << 2)) for k in cn if k != m]
    d = search([(1, m, 2)], extra=extra)
    expect(d, 0, 2, x)


def check_orphan_and_hole_neighbourhood():
    """One HOLE node inside a box: exactly the 8 cells sharing it lose their
    donor (the point has no other candidate grid, so it is an orphan); the
    other cells of the surrounding 4 x 4 x 4 block keep theirs. Fails if the
    hole is ignored or if FRINGE flags invalidate cells."""
    dims = (7, 7, 7)
    g = W.cartesian_grid(dims)
    h = 1.0 / 6
    i0, j0, k0 = 3, 2, 4
    fl = np.zeros(g.nodes, np.uint8)
    fl[i0 + 7 * (j0 + 7 * k0)] = 1 | (5 << 2)
    fl[i0 + 1 + 7 * (j0 + 7 * k0)] = FRINGE | (5 << 2)  # a buffer node beside it
    rng = np.random.default_rng(12)
    cells, pts = [], []
    for ck in range(k0 - 2, k0 + 2):
        for cj in range(j0 - 2, j0 + 2):
            for ci in range(i0 - 2, i0 + 2):
                s = rng.uniform(0.05, 0.95, 3)
                pts.append((np.array([ci, cj, ck]) + s) * h)
                cells.append((ci, cj, ck))
    d = search_points(g, np.array(pts), donor_flags=fl)
    for n, (ci, cj, ck) in enumerate(cells):
        touches = ci in (i0 - 1, i0) and cj in (j0 - 1, j0) and ck in (k0 - 1, k0)
        if touches:
            assert d["donor_grid"][n] == -1 and d["donor_cell"][n] == -1 and np.all(np.isnan(d["s"][n]))
        else:
            assert d["donor_grid"][n] == 0 and d["donor_cell"][n] == cell_index(dims, 0, ci, cj, ck)
    assert sum(d["donor_grid"] < 0) == 8


def check_invalid_everywhere_is_orphan():
    """A background node cut by overset 1, inside overset 1 only, whose
    containing cell there has a HOLE corner: no candidate remains, so it is
    an orphan. Fails if an invalid cell is accepted or if the search falls
    back to some other cell of the same grid."""
    # a background node inside box 1 but outside box 2
    cand = [m for m in range(GRIDS[0].nodes)
            if closed_form(1, world(0, m)) is not None and closed_form(2, world(0, m)) is None
            and closed_form(1, world(0, m))[2] >= 1e-3]
    m = cand[len(cand) // 2]
    cell1 = closed_form(1, world(0, m))[0]
    d = search([(0, m, 1)], extra=[(1, corners(1, cell1)[3], 1 | (3 << 2))])
    assert d["donor_grid"][0] == -1 and d["donor_cell"][0] == -1
    d = search([(0, m, 1)])
    expect(d, 0, 1, world(0, m))


PINS = [check_priority, check_hole_corner_in_donor_grid, check_fringe_corners_valid,
        check_orphan_and_hole_neighbourhood, check_invalid_everywhere_is_orphan]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin_holds(pin):
    pin()


# ------------------------------------------------------------------ planted mistakes
# (label, text of the oracle source, replacement, the pins that must fail)
_CAUSE = "if (cause != CAUSE_BOUNDARY && cause != A && cause < ngrids) out[n++] = cause;"
_BG = "if (A != 0 && !(n == 1 && out[0] == 0)) out[n++] = 0;"
MUTANTS = [
    ("background_before_cause", _CAUSE + "\n    " + _BG,
     "if (A != 0) out[n++] = 0;\n    if (cause != CAUSE_BOUNDARY && cause != A && cause < ngrids && cause != 0) "
     "out[n++] = cause;", ["check_priority"]),
    ("cause_ignored", _CAUSE, "(void)cause;", ["check_priority"]),
    ("query_grid_flags", "const uint8_t *fl = flags + node_off[B];", "const uint8_t *fl = flags + node_off[A];",
     ["check_hole_corner_in_donor_grid", "check_fringe_corners_valid"]),
    ("fringe_corner_rejected", "if ((fl[nd[c]] & 3) == ST_HOLE) return 0;",
     "if ((fl[nd[c]] & 3) != ST_FIELD) return 0;",
     ["check_fringe_corners_valid", "check_orphan_and_hole_neighbourhood"]),
    ("hole_cause_bits_not_masked", "if ((fl[nd[c]] & 3) == ST_HOLE) return 0;",
     "if (fl[nd[c]] == ST_HOLE) return 0;",
     ["check_hole_corner_in_donor_grid", "check_orphan_and_hole_neighbourhood",
      "check_invalid_everywhere_is_orphan"]),
    ("hole_ignored", "if ((fl[nd[c]] & 3) == ST_HOLE) return 0;", "(void)fl;",
     ["check_hole_corner_in_donor_grid", "check_orphan_and_hole_neighbourhood",
      "check_invalid_everywhere_is_orphan"]),
]


@pytest.mark.parametrize("label,old,new,failing", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(label, old, new, failing, tmp_path, monkeypatch):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "overset_oracle.c")).read()
    assert src.count(old) == 1, f"mutation target of {label} not found once in the oracle source"
    path = tmp_path / f"{label}.c"
    path.write_text(src.replace(old, new))
    lib = oracle.bind(ctypes.CDLL(oracle.build(force=True, src=str(path), out=str(tmp_path / f"{label}.so"))))
    monkeypatch.setattr(oracle, "_lib", lib)
    pins = {p.__name__: p for p in PINS}
    for name in failing:
        with pytest.raises(AssertionError):
            pins[name]()

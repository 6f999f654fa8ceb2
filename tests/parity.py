"""Comparison of one GPU step against the CPU oracle (not collected by pytest).

Bar (per step):
  * flags of every node: bit-exact (state and cause);
  * the ordered query list and its count: bit-exact;
  * the orphan set: bit-exact;
  * donor (grid, cell) of every query whose oracle margin is >= `gate`
    (1e-3 of a cell face in natural coordinates): bit-exact;
  * every other GPU donor must be valid: the oracle's Newton in the GPU's cell
    gives s in [-1e-9, 1 + 1e-9]^3 and no corner of it is a hole; and it must
    lie in the oracle's donor grid, unless the two sides chose different
    grids because the point lies within 1e-9 (in natural coordinates) of the
    outer boundary of the one that comes first in the query's candidate order
    (Sec. 2.4 item 1: cause grid, background, ascending ids);
  * s on gated queries within `s_tol`;
  * interpolated values where donors agree: per field, max |gpu - oracle| <=
    value_rtol * max |oracle| (normwise), and an identically zero field stays 0.
"""
import numpy as np

import oracle


def _corner_nodes(dims, periodic, cell):
    ni, nj, nk = dims
    nci = ni if periodic & 1 else ni - 1
    ncj = nj if periodic & 2 else nj - 1
    ci, cj, ck = cell % nci, (cell // nci) % ncj, cell // (nci * ncj)
    out = []
    for c in range(8):
        i, j, k = ci + (c & 1), cj + ((c >> 1) & 1), ck + ((c >> 2) & 1)
        i, j, k = i % ni, j % nj, k % nk
        out.append(i + ni * (j + nj * k))
    return out


def _cell_ijk(dims, periodic, cell):
    ni, nj, nk = dims
    nc = (ni if periodic & 1 else ni - 1, nj if periodic & 2 else nj - 1, nk if periodic & 4 else nk - 1)
    return (cell % nc[0], (cell // nc[0]) % nc[1], cell // (nc[0] * nc[1])), nc


def _on_outer_boundary(grid, cell, s, tol=1e-9):
    """Whether natural coordinates s in `cell` lie within tol of a face of
    the cell that is part of the grid's outer (non-periodic) boundary."""
    (ci, cj, ck), nc = _cell_ijk(grid.dims, grid.periodic, cell)
    for d, c in enumerate((ci, cj, ck)):
        if grid.periodic & (1 << d):
            continue
        if (c == 0 and s[d] <= tol) or (c == nc[d] - 1 and s[d] >= 1 - tol):
            return True
    return False


def candidate_order(ngrids, A, cause):
    """Candidate donor grids of a query of grid A with flag cause `cause`."""
    out = []
    if cause != oracle.CAUSE_BOUNDARY and cause != A and cause < ngrids:
        out.append(cause)
    if A != 0 and 0 not in out:
        out.append(0)
    out += [g for g in range(ngrids) if g != A and g not in out]
    return out


def query_world(o: "oracle.Oracle", poses, q_grid, q_node):
    x = np.empty((len(q_grid), 3))
    for g in np.unique(q_grid):
        sel = q_grid == g
        w = o.transform(poses[g], int(g), q_node[sel])
        x[sel] = np.stack(w, 1)
    return x


def compare(o: "oracle.Oracle", poses, ref: dict, gpu: dict, value_rtol: float, s_tol: float = 1e-12,
            gate: float = 1e-3, qx_tol: float = 1e-14) -> dict:
    poses = np.asarray(poses).reshape(o.ng, 12)
    bad = np.flatnonzero(ref["flags"] != gpu["flags"])
    assert bad.size == 0, f"{bad.size} flag mismatches, first at {bad[:5]}: oracle {ref['flags'][bad[:5]]} gpu {gpu['flags'][bad[:5]]}"
    n = len(ref["q_grid"])
    assert gpu["count"] == n, (gpu["count"], n)
    assert np.array_equal(gpu["q_grid"], ref["q_grid"]) and np.array_equal(gpu["q_node"], ref["q_node"])
    if n:
        # transform: frame centre + GPU offset against the oracle's inertial position
        xw = query_world(o, poses, ref["q_grid"], ref["q_node"])
        dx = np.abs(gpu["qx"] + poses[ref["q_grid"], 9:] - xw).max()
        assert dx <= qx_tol, f"transform differs by {dx:.3e}"
    orph_r = ref["donor_grid"] < 0
    orph_g = gpu["donor_grid"] < 0
    diff = np.flatnonzero(orph_r != orph_g)
    assert diff.size == 0, f"orphan sets differ at {diff[:10]} (oracle margin {ref['margin'][diff[:10]]})"
    gated = ~orph_r & (ref["margin"] >= gate)
    dm = np.flatnonzero(gated & ((gpu["donor_grid"] != ref["donor_grid"]) | (gpu["donor_cell"] != ref["donor_cell"])))
    assert dm.size == 0, (f"{dm.size} gated donors differ, first {dm[:5]}: oracle {ref['donor_grid'][dm[:5]]}/"
                          f"{ref['donor_cell'][dm[:5]]} gpu {gpu['donor_grid'][dm[:5]]}/{gpu['donor_cell'][dm[:5]]}")
    # validity of the other GPU donors
    near = ~orph_r & ~gated
    other = np.flatnonzero(near & ((gpu["donor_grid"] != ref["donor_grid"]) | (gpu["donor_cell"] != ref["donor_cell"])))
    if other.size:
        xw = query_world(o, poses, gpu["q_grid"][other], gpu["q_node"][other])
        for t, q in enumerate(other):
            g, cell = int(gpu["donor_grid"][q]), int(gpu["donor_cell"][q])
            R, c = poses[g, :9].reshape(3, 3), poses[g, 9:]
            xi = R.T @ (xw[t] - c)
            ok, s = o.cell_coords(g, cell, xi)
            assert ok and np.all(s >= -1e-9) and np.all(s <= 1 + 1e-9), (q, g, cell, s)
            gr = o.grids[g]
            nodes = _corner_nodes(gr.dims, gr.periodic, cell)
            assert np.all((ref["flags"][o.node_off[g] + np.array(nodes)] & 3) != oracle.ST_HOLE), (q, g, cell)
            rg = int(ref["donor_grid"][q])
            if g != rg:
                # a different grid only where the point sits on the outer
                # boundary of the grid that comes first for this query
                A = int(ref["q_grid"][q])
                order = candidate_order(o.ng, A, int(ref["flags"][o.node_off[A] + ref["q_node"][q]]) >> 2)
                if order.index(g) < order.index(rg):
                    first, fcell, fs = g, cell, s
                else:
                    first, fcell, fs = rg, int(ref["donor_cell"][q]), ref["s"][q]
                assert _on_outer_boundary(o.grids[first], fcell, fs), (
                    f"query {q}: GPU donor grid {g}, oracle {rg}, and the point is not on the outer boundary of "
                    f"grid {first} (cell {fcell}, s {fs})")
    if gated.any():
        ds = np.abs(gpu["s"][gated] - ref["s"][gated]).max()
        assert ds <= s_tol, f"s differs by {ds}"
    same = ~orph_r & (gpu["donor_grid"] == ref["donor_grid"]) & (gpu["donor_cell"] == ref["donor_cell"])
    errs = []
    if "values" in gpu and same.any():
        for f in range(ref["values"].shape[0]):
            r = ref["values"][f][same]
            v = gpu["values"][f][same]
            scale = np.abs(r).max()
            if scale == 0.0:
                assert np.all(v == 0.0), f"field {f}: expected exact zeros"
                errs.append(0.0)
                continue
            e = np.abs(v - r).max() / scale
            errs.append(float(e))
            assert e <= value_rtol, f"field {f}: normwise relative error {e:.3e} > {value_rtol:.1e}"
    other_grid = int(np.sum(gpu["donor_grid"][other] != ref["donor_grid"][other])) if other.size else 0
    return {"queries": n, "orphans": int(orph_r.sum()), "gated": int(gated.sum()), "near": int(near.sum()),
            "near_other_cell": int(other.size), "near_other_grid": other_grid, "value_err": errs}

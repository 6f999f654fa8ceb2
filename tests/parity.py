"""Comparison of one GPU step against the CPU oracle (not collected by pytest).

Bar (per step):
  * flags of every node: bit-exact (state and cause);
  * the ordered query list and its count: bit-exact;
  * the orphan set: bit-exact;
  * donor (grid, cell) of every query whose oracle margin is >= `gate`
    (1e-3 of a cell face in natural coordinates): bit-exact;
  * every other GPU donor must be valid: the oracle's Newton in the GPU's cell
    gives s in [-1e-9, 1 + 1e-9]^3 and no corner of it is a hole;
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
    return {"queries": n, "orphans": int(orph_r.sum()), "gated": int(gated.sum()), "near": int(near.sum()),
            "near_other_cell": int(other.size), "value_err": errs}

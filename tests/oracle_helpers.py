"""Helpers to drive the CPU oracle on hand-made inputs (not collected by pytest)."""
import numpy as np

import oracle
import workloads as W


def points_grid(pts, name="points"):
    """A 'grid' whose nodes are arbitrary world points (dims n x 1 x 1)."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    return W.Grid(name, (len(pts), 1, 1), 0, pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy())


def search_points(donor, pts, donor_pose=None, donor_flags=None, exhaustive=False):
    """Oracle donor search of world points `pts` in grid `donor` placed at
    `donor_pose`. The points form grid 1 (flag: fringe, boundary cause), so
    the donor grid is their only candidate."""
    pg = points_grid(pts)
    o = oracle.Oracle([donor, pg], nf=0)
    poses = np.stack([W.IDENTITY_POSE if donor_pose is None else donor_pose, W.IDENTITY_POSE])
    flags = np.zeros(o.total_nodes, dtype=np.uint8)
    if donor_flags is not None:
        flags[: donor.nodes] = donor_flags
    flags[donor.nodes:] = oracle.ST_FRINGE | (oracle.CAUSE_BOUNDARY << 2)
    n = pg.nodes
    d = o.donor_search(poses, flags, np.ones(n, np.int32), np.arange(n, dtype=np.int32), exhaustive=exhaustive)
    d["oracle"] = o
    d["flags"] = flags
    return d


def interp_points(donor, pts, fields_donor, donor_pose=None):
    """Search and interpolate `fields_donor` ([nf, donor.nodes]) at `pts`."""
    d = search_points(donor, pts, donor_pose)
    o = d["oracle"]
    nf = fields_donor.shape[0]
    fields = np.zeros((nf, o.total_nodes))
    fields[:, : donor.nodes] = fields_donor
    vals = o.interp(fields, d["donor_grid"], d["donor_cell"], d["s"])
    return d, vals


def cell_index(dims, periodic, ci, cj, ck):
    ni, nj, nk = dims
    nci = ni if periodic & 1 else ni - 1
    ncj = nj if periodic & 2 else nj - 1
    return ci + nci * (cj + ncj * ck)

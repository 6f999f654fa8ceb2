"""CPU FP64 oracle for the overset grid-assembly path.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package. The product path
(the HIP library and its binding) never imports, links or runs it, and the
two share no code. The arithmetic lives in ``overset_oracle.c`` (plain C,
FP64, ``-ffp-contract=off``); this module only marshals numpy arrays.

Each stage follows a passage of Hedayat & Borazjani, arXiv:1910.09315:
transform (Sec. 2.1), hole cutting (Sec. 2.2.2), query points (Sec. 2.2.3,
Alg. 1), donor search by control cells and brute force (Sec. 2.2.5, Alg. 3),
donor priority (Sec. 2.4 item 1), trilinear interpolation (Sec. 2.2.6),
velocities in the receiver's frame (Sec. 2.3), the interpolation matrix and
its application (Sec. 2.2.6 second option, Alg. 4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "overset_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboverset_oracle.so")

ST_FIELD, ST_HOLE, ST_FRINGE = 0, 1, 2
CAUSE_BOUNDARY = 63

_lib = None
_P = ctypes.c_void_p


def build(force: bool = True, src: str = _SRC, out: str = LIB_PATH) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP); `src` and
    `out` default to this package's source and library."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                        "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"], check=True)
        os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = bind(ctypes.CDLL(LIB_PATH))
    return _lib


def bind(L):
    """Declare the argument and result types of the oracle's entry points on
    the loaded library `L` (also used by tests that load a variant build)."""
    L.orc_holecut.restype = ctypes.c_double
    L.orc_holecut.argtypes = [ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_mesh_inside.restype = ctypes.c_double
    L.orc_mesh_inside.argtypes = [_P, ctypes.c_int64, ctypes.c_int64, _P, _P]
    L.orc_fringe.restype = None
    L.orc_fringe.argtypes = [ctypes.c_int, _P, _P, ctypes.c_int, _P, _P]
    L.orc_compact.restype = ctypes.c_int64
    L.orc_compact.argtypes = [ctypes.c_int, _P, _P, _P, _P, ctypes.c_int64]
    L.orc_bins_build.restype = _P
    L.orc_bins_build.argtypes = [_P, _P, _P, _P]
    L.orc_bins_free.restype = None
    L.orc_bins_free.argtypes = [_P]
    L.orc_bins_entries.restype = ctypes.c_int64
    L.orc_bins_entries.argtypes = [_P]
    L.orc_donor_search.restype = None
    L.orc_donor_search.argtypes = [ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int,
                                   ctypes.c_int64, _P, _P, _P, _P, _P, _P]
    L.orc_cell_coords.restype = ctypes.c_int
    L.orc_cell_coords.argtypes = [_P, _P, _P, _P, ctypes.c_int64, _P, _P]
    L.orc_interp.restype = None
    L.orc_interp.argtypes = [ctypes.c_int, _P, _P, ctypes.c_int64, ctypes.c_int, _P, ctypes.c_int64,
                             _P, _P, _P, _P]
    L.orc_transform.restype = None
    L.orc_transform.argtypes = [_P, _P, _P, _P, _P, ctypes.c_int64, _P, _P, _P]
    L.orc_weights.restype = None
    L.orc_weights.argtypes = [_P, _P]
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_set_threads.restype = None
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_frame_velocity.restype = None
    L.orc_frame_velocity.argtypes = [_P, ctypes.c_int64, _P, _P, _P]
    L.orc_interp_matrix.restype = None
    L.orc_interp_matrix.argtypes = [_P, _P, ctypes.c_int64, _P, _P, _P, _P, _P]
    L.orc_matrix_apply.restype = None
    L.orc_matrix_apply.argtypes = [ctypes.c_int64, _P, _P, ctypes.c_int, ctypes.c_int64, _P, _P]
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Thread count of the oracle's later parallel loops (for timing)."""
    lib().orc_set_threads(int(n))


class Oracle:
    """Stage-by-stage oracle over one workload's grids (see `workloads`)."""

    def __init__(self, grids, nf: int):
        self.grids = grids
        self.nf = nf
        self.ng = len(grids)
        self.dims = np.array([[*g.dims, g.periodic] for g in grids], dtype=np.int32).ravel()
        self.outer = np.array([g.outer for g in grids], dtype=np.int32).ravel()
        self.blank_kind = np.array([g.blank_kind for g in grids], dtype=np.int32)
        self.blank_prm = np.stack([g.blank_prm8() for g in grids]).ravel()
        self.node_off = np.zeros(self.ng + 1, dtype=np.int64)
        self.node_off[1:] = np.cumsum([g.nodes for g in grids])
        self._X = [np.ascontiguousarray(g.X, dtype=np.float64) for g in grids]
        self._Y = [np.ascontiguousarray(g.Y, dtype=np.float64) for g in grids]
        self._Z = [np.ascontiguousarray(g.Z, dtype=np.float64) for g in grids]
        self.Xp = np.array([a.ctypes.data for a in self._X], dtype=np.uint64)
        self.Yp = np.array([a.ctypes.data for a in self._Y], dtype=np.uint64)
        self.Zp = np.array([a.ctypes.data for a in self._Z], dtype=np.uint64)
        self._bins = [None] * self.ng
        # triangulated blank surfaces (ray-parity hole cut), per grid
        self._mesh = [np.ascontiguousarray(getattr(g, "blank_mesh", None), dtype=np.float64).reshape(-1)
                      if getattr(g, "blank_mesh", None) is not None else None for g in grids]
        self.mesh_ptr = np.array([m.ctypes.data if m is not None else 0 for m in self._mesh], dtype=np.uint64)
        self.mesh_ntri = np.array([m.size // 9 if m is not None else 0 for m in self._mesh], dtype=np.int64)

    @property
    def total_nodes(self) -> int:
        return int(self.node_off[-1])

    def __del__(self):
        try:
            for b in self._bins:
                if b:
                    lib().orc_bins_free(b)
        except Exception:
            pass

    def bins(self, g: int):
        if self._bins[g] is None:
            self._bins[g] = lib().orc_bins_build(_ptr(self.dims[4 * g:4 * g + 4]), _ptr(self._X[g]),
                                                 _ptr(self._Y[g]), _ptr(self._Z[g]))
        return self._bins[g]

    def transform(self, pose, g: int, idx=None):
        pose = np.ascontiguousarray(pose, dtype=np.float64)
        n = self.grids[g].nodes if idx is None else len(idx)
        out = [np.empty(n) for _ in range(3)]
        ip = None if idx is None else _ptr(np.ascontiguousarray(idx, dtype=np.int32))
        lib().orc_transform(_ptr(pose), _ptr(self._X[g]), _ptr(self._Y[g]), _ptr(self._Z[g]), ip, n,
                            _ptr(out[0]), _ptr(out[1]), _ptr(out[2]))
        return out

    def holecut(self, poses):
        poses = np.ascontiguousarray(poses, dtype=np.float64).reshape(self.ng, 12)
        flags = np.empty(self.total_nodes, dtype=np.uint8)
        gap = lib().orc_holecut(self.ng, _ptr(self.dims), _ptr(self.Xp), _ptr(self.Yp), _ptr(self.Zp),
                                _ptr(self.blank_kind), _ptr(self.blank_prm), _ptr(poses),
                                _ptr(self.node_off), _ptr(flags), _ptr(self.mesh_ptr), _ptr(self.mesh_ntri))
        return flags, gap

    def fringe(self, flags, nf=None):
        nf = self.nf if nf is None else nf
        lib().orc_fringe(self.ng, _ptr(self.dims), _ptr(self.outer), nf, _ptr(self.node_off), _ptr(flags))
        return flags

    def compact(self, flags):
        n = int(np.count_nonzero((flags & 3) == ST_FRINGE))
        qg = np.empty(max(n, 1), dtype=np.int32)
        qn = np.empty(max(n, 1), dtype=np.int32)
        cnt = lib().orc_compact(self.ng, _ptr(self.node_off), _ptr(flags), _ptr(qg), _ptr(qn), n)
        assert cnt == n
        return qg[:n].copy(), qn[:n].copy()

    def donor_search(self, poses, flags, q_grid, q_node, exhaustive=False):
        poses = np.ascontiguousarray(poses, dtype=np.float64).reshape(self.ng, 12)
        nq = len(q_grid)
        q_grid = np.ascontiguousarray(q_grid, dtype=np.int32)
        q_node = np.ascontiguousarray(q_node, dtype=np.int32)
        if exhaustive:
            bins = np.zeros(self.ng, dtype=np.uint64)
        else:
            bins = np.array([self.bins(g) for g in range(self.ng)], dtype=np.uint64)
        dg = np.empty(max(nq, 1), dtype=np.int32)
        dc = np.empty(max(nq, 1), dtype=np.int32)
        s = np.empty((max(nq, 1), 3), dtype=np.float64)
        mg = np.empty(max(nq, 1), dtype=np.float64)
        lib().orc_donor_search(self.ng, _ptr(self.dims), _ptr(self.Xp), _ptr(self.Yp), _ptr(self.Zp),
                               _ptr(self.node_off), _ptr(flags), _ptr(poses), _ptr(bins), int(exhaustive),
                               nq, _ptr(q_grid), _ptr(q_node), _ptr(dg), _ptr(dc), _ptr(s), _ptr(mg))
        return {"donor_grid": dg[:nq], "donor_cell": dc[:nq], "s": s[:nq], "margin": mg[:nq]}

    def cell_coords(self, g, cell, xi):
        s = np.empty(3)
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        ok = lib().orc_cell_coords(_ptr(self.dims[4 * g:4 * g + 4]), _ptr(self._X[g]), _ptr(self._Y[g]),
                                   _ptr(self._Z[g]), int(cell), _ptr(xi), _ptr(s))
        return bool(ok), s

    def interp(self, fields, donor_grid, donor_cell, s):
        fields = np.ascontiguousarray(fields, dtype=np.float64)
        nfields = fields.shape[0]
        nq = len(donor_grid)
        out = np.full((nfields, max(nq, 1)), np.nan)
        lib().orc_interp(self.ng, _ptr(self.dims), _ptr(self.node_off), self.total_nodes, nfields,
                         _ptr(fields), nq, _ptr(np.ascontiguousarray(donor_grid, dtype=np.int32)),
                         _ptr(np.ascontiguousarray(donor_cell, dtype=np.int32)),
                         _ptr(np.ascontiguousarray(s, dtype=np.float64)), _ptr(out))
        return out[:, :nq]

    def step(self, poses, fields, exhaustive=False):
        """All stages of one time step; returns every intermediate result."""
        flags, gap = self.holecut(poses)
        holes = flags.copy()
        self.fringe(flags)
        qg, qn = self.compact(flags)
        d = self.donor_search(poses, flags, qg, qn, exhaustive=exhaustive)
        vals = self.interp(fields, d["donor_grid"], d["donor_cell"], d["s"])
        return {"holecut_flags": holes, "flags": flags, "min_gap": gap, "q_grid": qg, "q_node": qn,
                **d, "values": vals}


def mesh_inside(tri, points):
    """Ray-parity inside test of points [n, 3] against the closed
    triangulated surface tri [ntri, 3, 3] (body frame). Returns (inside
    bool [n], smallest crossing gap)."""
    t = np.ascontiguousarray(tri, dtype=np.float64).reshape(-1)
    p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(p), dtype=np.uint8)
    gap = lib().orc_mesh_inside(_ptr(t), t.size // 9, len(p), _ptr(p), _ptr(out))
    return out.astype(bool), gap


def frame_velocity(poses, q_grid, donor_grid, values):
    """Velocity components (fields 0..2 of `values`, [nfields, nq]) turned
    from each donor's frame into its receiver's frame (Sec. 2.3); returns a
    new array."""
    out = np.ascontiguousarray(values, dtype=np.float64).copy()
    nq = out.shape[1]
    lib().orc_frame_velocity(_ptr(np.ascontiguousarray(poses, dtype=np.float64).reshape(-1)), nq,
                             _ptr(np.ascontiguousarray(q_grid, dtype=np.int32)),
                             _ptr(np.ascontiguousarray(donor_grid, dtype=np.int32)), _ptr(out))
    return out


def interp_matrix(o, donor_grid, donor_cell, s):
    """The interpolation matrix of Alg. 4 for Oracle `o`: (cols [nq, 8] int64
    global node indices, -1 for no donor; vals [nq, 8] weights)."""
    nq = len(donor_grid)
    cols = np.empty((max(nq, 1), 8), dtype=np.int64)
    vals = np.empty((max(nq, 1), 8))
    lib().orc_interp_matrix(_ptr(o.dims), _ptr(o.node_off), nq,
                            _ptr(np.ascontiguousarray(donor_grid, dtype=np.int32)),
                            _ptr(np.ascontiguousarray(donor_cell, dtype=np.int32)),
                            _ptr(np.ascontiguousarray(s, dtype=np.float64)), _ptr(cols), _ptr(vals))
    return cols[:nq], vals[:nq]


def matrix_apply(cols, vals, x):
    """y = M x for the rows of (cols, vals) and x [nrhs, total_nodes]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    nrhs, total = x.shape
    nq = cols.shape[0]
    y = np.empty((nrhs, max(nq, 1)))
    lib().orc_matrix_apply(nq, _ptr(np.ascontiguousarray(cols, dtype=np.int64)),
                           _ptr(np.ascontiguousarray(vals, dtype=np.float64)), nrhs, total, _ptr(x), _ptr(y))
    return y[:, :nq]


def weights(s):
    w = np.empty(8)
    lib().orc_weights(_ptr(np.ascontiguousarray(s, dtype=np.float64)), _ptr(w))
    return w

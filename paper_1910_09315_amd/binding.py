"""ctypes binding of liboverset.so (include/overset.h).

Argument marshalling only: every stage runs in the library's HIP kernels.
Device buffers are torch tensors on a ROCm device; their data pointers and
the current torch stream (a hipStream_t) are handed to the C ABI. If the
library has not been built, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboverset.so")

OV_FP64, OV_MIXED = 0, 1
OV_BLANK_NONE, OV_BLANK_CYL, OV_BLANK_SPHERE, OV_BLANK_ELLIPSOID = 0, 1, 2, 3
OV_BLANK_NONE, OV_BLANK_CYL, OV_BLANK_SPHERE, OV_BLANK_ELLIPSOID, OV_BLANK_MESH = 0, 1, 2, 3, 4
OV_STATE_FIELD, OV_STATE_HOLE, OV_STATE_FRINGE = 0, 1, 2
OV_CAUSE_BOUNDARY = 63
OV_Q_ORPHAN, OV_Q_FOUND, OV_Q_FALLBACK, OV_Q_FP64_FIXED = 0, 1, 2, 4
OV_DEV_CAPACITY, OV_DEV_WALK_LIMIT, OV_DEV_NONFINITE = 1, 2, 4
# work counters (OV_STAT_*)
STAT = {"holecut_nodes_read": 0, "holecut_calls": 1, "search_cells": 2, "newton_iters": 3, "scan_candidates": 4,
        "back_calls": 5, "flag_bytes_written": 6, "base_bytes_read": 7, "flag_starts": 8}
OV_STAT_COUNT = 9
OPT = {"warm": 1, "max_walk": 2, "search_block": 3, "interp_block": 4, "holecut_block": 5,
       "holecut_npt": 6, "persist": 7, "holecut_cull": 8, "holecut_npl": 9,
       "back_fused": 10, "back_blocks": 11, "back_block": 12, "field_layout": 13,
       "frame_velocity": 14, "back_queue": 15, "back_xcd": 16, "holecut_list": 17}

EXPORTS = ["ov_ctx_create", "ov_ctx_destroy", "ov_last_error", "ov_grid_add", "ov_grid_set_blank_mesh",
           "ov_finalize", "ov_num_grids",
           "ov_total_nodes", "ov_node_offsets", "ov_set_option", "ov_reset_history", "ov_status_fetch",
           "ov_stats_fetch", "overset_status_fetch", "overset_last_error",
           "overset_holecut", "overset_fringe_compact", "overset_fringe_compact_noalloc", "overset_transform", "overset_donor_search",
           "overset_interp", "overset_frame_velocity", "overset_interp_matrix", "overset_interp_apply",
           "ov_pipe_create1", "ov_pipe_create", "ov_pipe_create3", "ov_pipe_use_graphs",
           "ov_pipe_submit",
           "ov_pipe_submit_many", "ov_pipe_set_threads", "ov_pipe_set_by_step", "ov_pipe_join", "ov_pipe_set_timing", "ov_pipe_set_timing_mode", "ov_pipe_stage_times",
           "ov_pipe_destroy"]

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_lib = None


class OversetError(RuntimeError):
    pass


class StepBuffersC(ctypes.Structure):
    """ov_step_buffers (include/overset.h)."""
    _fields_ = [("flags", _P), ("q_grid", _P), ("q_node", _P), ("d_count", _P), ("qx", _P),
                ("donor_grid", _P), ("donor_cell", _P), ("s", _P), ("status", _P), ("out", _P),
                ("capacity", _I64)]


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OversetError(f"{path} is missing: build it with paper_1910_09315_amd.build.build()")
    L = ctypes.CDLL(path)
    sig = {
        "ov_ctx_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int]),
        "ov_ctx_destroy": (ctypes.c_int, [_P]),
        "ov_last_error": (ctypes.c_char_p, [_P]),
        "ov_grid_add": (ctypes.c_int, [_P, _I32, _I32, _I32, ctypes.c_uint32, _P, _P, _P, _I32, _P, _P, _P]),
        "ov_grid_set_blank_mesh": (ctypes.c_int, [_P, _I32, _P, _I64]),
        "ov_finalize": (ctypes.c_int, [_P, _P]),
        "ov_num_grids": (_I32, [_P]),
        "ov_total_nodes": (_I64, [_P]),
        "ov_node_offsets": (ctypes.c_int, [_P, _P]),
        "ov_set_option": (ctypes.c_int, [_P, _I32, _I64]),
        "ov_reset_history": (ctypes.c_int, [_P, _P]),
        "ov_status_fetch": (ctypes.c_int, [_P, _P, _P]),
        "ov_stats_fetch": (ctypes.c_int, [_P, _P, _P]),
        "overset_status_fetch": (ctypes.c_int, [_P, _P, _P]),
        "overset_last_error": (ctypes.c_char_p, [_P]),
        "overset_holecut": (ctypes.c_int, [_P, _P, _P, _P]),
        "overset_fringe_compact": (ctypes.c_int, [_P, _I32, _P, _P, _P, _I64, _P, _P]),
        "overset_fringe_compact_noalloc": (ctypes.c_int, [_P, _I32, _P, _P, _P, _I64, _P, _P]),
        "overset_transform": (ctypes.c_int, [_P, _P, _P, _P, _P, _I64, _P, _P]),
        "overset_donor_search": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _P]),
        "overset_interp": (ctypes.c_int, [_P, _P, _P, _P, _P, _I64, _P, _P, _P]),
        "overset_frame_velocity": (ctypes.c_int, [_P, _P, _P, _P, _P, _I64, _P, _P]),
        "overset_interp_matrix": (ctypes.c_int, [_P, _P, _P, _P, _P, _I64, _P, _P, _P]),
        "overset_interp_apply": (ctypes.c_int, [_P, _P, _P, _P, _I64, _P, _I32, _I32, _P, _P]),
        "ov_pipe_create": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _I32, ctypes.POINTER(_P)]),
        "ov_pipe_create3": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _P, _I32, ctypes.POINTER(_P)]),
        "ov_pipe_create1": (ctypes.c_int, [_P, _I32, _P, _P, _P, _I32, ctypes.POINTER(_P)]),
        "ov_pipe_use_graphs": (ctypes.c_int, [_P, _I32]),
        "ov_pipe_submit": (ctypes.c_int, [_P, _P, _P]),
        "ov_pipe_submit_many": (ctypes.c_int, [_P, _P, _I64, _I64, _P]),
        "ov_pipe_set_threads": (ctypes.c_int, [_P, _I32]),
        "ov_pipe_set_by_step": (ctypes.c_int, [_P, _I32]),
        "ov_pipe_join": (ctypes.c_int, [_P, _P]),
        "ov_pipe_set_timing": (ctypes.c_int, [_P, _I32, _I32]),
        "ov_pipe_set_timing_mode": (ctypes.c_int, [_P, _I32, _I32, _I32]),
        "ov_pipe_stage_times": (ctypes.c_int, [_P, _P, _I32, ctypes.POINTER(_I32)]),
        "ov_pipe_destroy": (ctypes.c_int, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(t):
    if t is None:
        return None
    return _P(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return _P(s.cuda_stream)


class Context:
    """Owns an ov_ctx (grids, control cells, warm-start history)."""

    def __init__(self, device: int = 0, precision: str = "fp64"):
        self.lib = load()
        self.precision = precision
        self.device = device
        h = _P()
        rc = self.lib.ov_ctx_create(ctypes.byref(h), device, OV_MIXED if precision == "mixed" else OV_FP64)
        if rc != 0:
            raise OversetError(f"ov_ctx_create failed ({rc})")
        self.h = h
        self._keep = []

    def check(self, rc: int, what: str):
        if rc != 0:
            msg = self.lib.overset_last_error(self.h)
            raise OversetError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "h", None):
            self.lib.ov_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def grid_add(self, dims, periodic, X, Y, Z, blank_kind=0, blank_prm=(), outer=(0,) * 6) -> int:
        prm = (ctypes.c_double * 8)(*([float(v) for v in blank_prm] + [0.0] * (8 - len(blank_prm))))
        out = (ctypes.c_int32 * 6)(*[int(v) for v in outer])
        gid = ctypes.c_int32()
        self._keep += [X, Y, Z]
        self.check(self.lib.ov_grid_add(self.h, int(dims[0]), int(dims[1]), int(dims[2]), int(periodic),
                                        _ptr(X), _ptr(Y), _ptr(Z), int(blank_kind), prm, out,
                                        ctypes.byref(gid)), "ov_grid_add")
        return gid.value

    def set_blank_mesh(self, grid: int, tri):
        """tri: [ntri, 3, 3] FP64 triangles of a closed surface (body frame); copied."""
        import numpy as np
        t = np.ascontiguousarray(tri, dtype=np.float64).reshape(-1)
        self.check(self.lib.ov_grid_set_blank_mesh(self.h, int(grid), t.ctypes.data_as(ctypes.c_void_p), t.size // 9),
                   "ov_grid_set_blank_mesh")

    def finalize(self, stream=None):
        self.check(self.lib.ov_finalize(self.h, _stream(stream)), "ov_finalize")

    def set_option(self, key: str, value: int):
        self.check(self.lib.ov_set_option(self.h, OPT[key], int(value)), f"ov_set_option({key})")

    def reset_history(self, stream=None):
        self.check(self.lib.ov_reset_history(self.h, _stream(stream)), "ov_reset_history")

    def status(self, stream=None) -> int:
        v = ctypes.c_int32()
        self.check(self.lib.overset_status_fetch(self.h, ctypes.byref(v), _stream(stream)), "overset_status_fetch")
        return v.value

    def stats(self, stream=None) -> list:
        """Work counters since the last fetch (OV_STAT_*, indices in STAT), then zeroed."""
        arr = (ctypes.c_int64 * OV_STAT_COUNT)()
        self.check(self.lib.ov_stats_fetch(self.h, arr, _stream(stream)), "ov_stats_fetch")
        return list(arr)

    def num_grids(self) -> int:
        return int(self.lib.ov_num_grids(self.h))

    def total_nodes(self) -> int:
        return int(self.lib.ov_total_nodes(self.h))

    def node_offsets(self):
        n = self.num_grids() + 1
        arr = (ctypes.c_int64 * n)()
        self.check(self.lib.ov_node_offsets(self.h, arr), "ov_node_offsets")
        return list(arr)


# ---------------------------------------------------------------- step calls (same names as the C ABI)
def overset_holecut(ctx: Context, poses, flags, stream=None):
    ctx.check(ctx.lib.overset_holecut(ctx.h, _ptr(poses), _ptr(flags), _stream(stream)), "overset_holecut")


def overset_fringe_compact(ctx: Context, nf, flags, q_grid, q_node, capacity, d_count, stream=None):
    ctx.check(ctx.lib.overset_fringe_compact(ctx.h, int(nf), _ptr(flags), _ptr(q_grid), _ptr(q_node),
                                             int(capacity), _ptr(d_count), _stream(stream)),
              "overset_fringe_compact")


def overset_fringe_compact_noalloc(ctx: Context, nf, flags, q_grid, q_node, capacity, d_count, stream=None):
    ctx.check(ctx.lib.overset_fringe_compact_noalloc(ctx.h, int(nf), _ptr(flags), _ptr(q_grid), _ptr(q_node),
                                                     int(capacity), _ptr(d_count), _stream(stream)),
              "overset_fringe_compact_noalloc")


def overset_transform(ctx: Context, poses, q_grid, q_node, d_count, capacity, qx, stream=None):
    ctx.check(ctx.lib.overset_transform(ctx.h, _ptr(poses), _ptr(q_grid), _ptr(q_node), _ptr(d_count),
                                        int(capacity), _ptr(qx), _stream(stream)), "overset_transform")


def overset_donor_search(ctx: Context, poses, flags, q_grid, q_node, qx, d_count, capacity, donor_grid,
                         donor_cell, s, status, stream=None):
    ctx.check(ctx.lib.overset_donor_search(ctx.h, _ptr(poses), _ptr(flags), _ptr(q_grid), _ptr(q_node), _ptr(qx),
                                           _ptr(d_count), int(capacity), _ptr(donor_grid), _ptr(donor_cell),
                                           _ptr(s), _ptr(status), _stream(stream)), "overset_donor_search")


def overset_interp(ctx: Context, donor_grid, donor_cell, s, d_count, capacity, fields, out, stream=None):
    ctx.check(ctx.lib.overset_interp(ctx.h, _ptr(donor_grid), _ptr(donor_cell), _ptr(s), _ptr(d_count),
                                     int(capacity), _ptr(fields), _ptr(out), _stream(stream)), "overset_interp")


def overset_frame_velocity(ctx: Context, poses, q_grid, donor_grid, d_count, capacity, out, stream=None):
    ctx.check(ctx.lib.overset_frame_velocity(ctx.h, _ptr(poses), _ptr(q_grid), _ptr(donor_grid), _ptr(d_count),
                                             int(capacity), _ptr(out), _stream(stream)), "overset_frame_velocity")


def overset_interp_matrix(ctx: Context, donor_grid, donor_cell, s, d_count, capacity, cols, vals, stream=None):
    ctx.check(ctx.lib.overset_interp_matrix(ctx.h, _ptr(donor_grid), _ptr(donor_cell), _ptr(s), _ptr(d_count),
                                            int(capacity), _ptr(cols), _ptr(vals), _stream(stream)),
              "overset_interp_matrix")


def overset_interp_apply(ctx: Context, cols, vals, d_count, capacity, x, nrhs, y, layout=0, stream=None):
    ctx.check(ctx.lib.overset_interp_apply(ctx.h, _ptr(cols), _ptr(vals), _ptr(d_count), int(capacity), _ptr(x),
                                           int(nrhs), int(layout), _ptr(y), _stream(stream)), "overset_interp_apply")


class NativePipe:
    """ov_pipe: the library's step executor. One stream and one buffer set
    (ov_pipe_create1), two streams (ov_pipe_create: front, back) and two
    buffer sets, or three streams (ov_pipe_create3: hole cut, fringe +
    compaction, back half) and three buffer sets."""

    def __init__(self, ctx: Context, nf: int, sets, fields, streams, max_timed: int = 0):
        self.ctx = ctx
        n = len(sets)
        if n not in (1, 2, 3) or len(streams) != n:
            raise OversetError("NativePipe: 1, 2 or 3 buffer sets, one stream per set")
        arr = (StepBuffersC * n)()
        for k, b in enumerate(sets):
            arr[k] = StepBuffersC(b.flags.data_ptr(), b.q_grid.data_ptr(), b.q_node.data_ptr(), b.d_count.data_ptr(),
                                  b.qx.data_ptr(), b.donor_grid.data_ptr(), b.donor_cell.data_ptr(),
                                  b.s.data_ptr(), b.status.data_ptr(), b.out.data_ptr(), b.capacity)
        self._keep = (sets, fields, streams)
        h = _P()
        st = [_P(x.cuda_stream) for x in streams]
        if n == 1:
            ctx.check(ctx.lib.ov_pipe_create1(ctx.h, int(nf), arr, _ptr(fields), st[0], int(max_timed),
                                              ctypes.byref(h)), "ov_pipe_create1")
        elif n == 2:
            ctx.check(ctx.lib.ov_pipe_create(ctx.h, int(nf), arr, _ptr(fields), st[0], st[1], int(max_timed),
                                             ctypes.byref(h)), "ov_pipe_create")
        else:
            ctx.check(ctx.lib.ov_pipe_create3(ctx.h, int(nf), arr, _ptr(fields), st[0], st[1], st[2],
                                              int(max_timed), ctypes.byref(h)), "ov_pipe_create3")
        self.h = h

    def use_graphs(self, on: bool = True):
        self.ctx.check(self.ctx.lib.ov_pipe_use_graphs(self.h, int(bool(on))), "ov_pipe_use_graphs")

    def submit(self, poses, count_out=None):
        self.ctx.check(self.ctx.lib.ov_pipe_submit(self.h, _ptr(poses), _ptr(count_out)), "ov_pipe_submit")

    def submit_many(self, poses, counts_out=None):
        """poses: device tensor [n, ngrids*12] (contiguous rows); counts_out: device int64[n] or None."""
        n, stride = int(poses.shape[0]), int(poses.stride(0))
        self.ctx.check(self.ctx.lib.ov_pipe_submit_many(self.h, _ptr(poses), stride, n, _ptr(counts_out)),
                       "ov_pipe_submit_many")

    def set_threads(self, on: bool = True):
        """Issue each stream's work of a multi-step submit from a host thread of its own."""
        self.ctx.check(self.ctx.lib.ov_pipe_set_threads(self.h, int(bool(on))), "ov_pipe_set_threads")

    def set_by_step(self, on: bool = True):
        """Run all stages of step t on stream t mod nsets (before the first submit)."""
        self.ctx.check(self.ctx.lib.ov_pipe_set_by_step(self.h, int(bool(on))), "ov_pipe_set_by_step")

    def join(self, stream=None):
        self.ctx.check(self.ctx.lib.ov_pipe_join(self.h, _stream(stream)), "ov_pipe_join")

    def set_timing(self, every: int, stage: int = 0, alone: bool = True):
        """Time stage `stage` (0 hole cut, 1 fringe + compaction, 2 back half)
        of the next step and every `every`-th step after it (0: stop); alone:
        the timed stage runs alone (else it keeps its place in the pipeline)."""
        self.ctx.check(self.ctx.lib.ov_pipe_set_timing_mode(self.h, int(every), int(stage), int(bool(alone))),
                       "ov_pipe_set_timing_mode")

    def stage_times(self, max_n: int):
        out = (ctypes.c_float * max(1, max_n))()
        n = _I32()
        self.ctx.check(self.ctx.lib.ov_pipe_stage_times(self.h, out, int(max_n), ctypes.byref(n)),
                       "ov_pipe_stage_times")
        return [out[i] for i in range(n.value)]

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.ov_pipe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

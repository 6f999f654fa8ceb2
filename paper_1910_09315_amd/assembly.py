"""Step driver: device buffers for one overset system and the five C-ABI
calls of a time step (hole cut, fringe compaction, transform, donor search,
interpolation), optionally replayed from a captured HIP graph.

Grids are any objects with ``dims``, ``periodic``, ``X``, ``Y``, ``Z``
(FP64 body-frame coordinates, i fastest), ``blank_kind``, ``blank_prm`` and
``outer``; grid 0 is the stationary background.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


class Assembly:
    def __init__(self, grids, nf: int, fields=None, precision: str = "fp64", capacity: int | None = None,
                 device: int = 0, options: dict | None = None):
        self.dev = torch.device("cuda", device)
        self.nf = int(nf)
        self.precision = precision
        self.dtype = torch.float32 if precision == "mixed" else torch.float64
        self.ctx = B.Context(device, precision)
        self.coords = []
        for g in grids:
            X = torch.as_tensor(np.ascontiguousarray(g.X, dtype=np.float64)).to(self.dev)
            Y = torch.as_tensor(np.ascontiguousarray(g.Y, dtype=np.float64)).to(self.dev)
            Z = torch.as_tensor(np.ascontiguousarray(g.Z, dtype=np.float64)).to(self.dev)
            self.coords.append((X, Y, Z))
            self.ctx.grid_add(g.dims, g.periodic, X, Y, Z, g.blank_kind, tuple(g.blank_prm), tuple(g.outer))
        self.ctx.finalize()
        for k, v in (options or {}).items():
            self.ctx.set_option(k, v)
        self.ngrids = len(grids)
        self.total = self.ctx.total_nodes()
        self.node_off = np.array(self.ctx.node_offsets(), dtype=np.int64)
        self.flags = torch.empty(self.total, dtype=torch.uint8, device=self.dev)
        self.d_count = torch.zeros(1, dtype=torch.int64, device=self.dev)
        self.fields = None
        if fields is not None:
            self.set_fields(fields)
        self.capacity = 0
        if capacity is not None:
            self.allocate(capacity)
        self.graph = None
        self.pose_slot = None

    # ------------------------------------------------------------ buffers
    def set_fields(self, fields):
        f = np.ascontiguousarray(fields, dtype=np.float64).reshape(4, self.total)
        self.fields = torch.as_tensor(f).to(self.dev).to(self.dtype).reshape(-1).contiguous()

    def allocate(self, capacity: int):
        cap = int(capacity)
        self.capacity = cap
        n = max(cap, 1)
        z = dict(device=self.dev)
        self.q_grid = torch.empty(n, dtype=torch.int32, **z)
        self.q_node = torch.empty(n, dtype=torch.int32, **z)
        self.qx = torch.empty(3 * n, dtype=self.dtype, **z)
        self.donor_grid = torch.empty(n, dtype=torch.int32, **z)
        self.donor_cell = torch.empty(n, dtype=torch.int32, **z)
        self.s = torch.empty(3 * n, dtype=self.dtype, **z)
        self.status = torch.empty(n, dtype=torch.int32, **z)
        self.out = torch.full((4 * n,), float("nan"), dtype=self.dtype, **z)

    def count_queries(self, poses) -> int:
        """Hole cut + fringe compaction with capacity 0: returns the count."""
        p = self.as_poses(poses)
        B.overset_holecut(self.ctx, p, self.flags)
        B.overset_fringe_compact(self.ctx, self.nf, self.flags, None, None, 0, self.d_count)
        torch.cuda.synchronize(self.dev)
        self.ctx.status()  # clears the capacity bit this probe sets
        return int(self.d_count.item())

    def as_poses(self, poses):
        if isinstance(poses, torch.Tensor) and poses.is_cuda:
            return poses.reshape(-1)
        return torch.as_tensor(np.ascontiguousarray(poses, dtype=np.float64).reshape(-1)).to(self.dev)

    # ------------------------------------------------------------ the step
    def step(self, poses, stream=None):
        """One time step on the current stream; nothing synchronises."""
        p = self.as_poses(poses)
        cap = self.capacity
        B.overset_holecut(self.ctx, p, self.flags, stream)
        B.overset_fringe_compact(self.ctx, self.nf, self.flags, self.q_grid, self.q_node, cap, self.d_count, stream)
        B.overset_transform(self.ctx, p, self.q_grid, self.q_node, self.d_count, cap, self.qx, stream)
        B.overset_donor_search(self.ctx, p, self.flags, self.q_grid, self.q_node, self.qx, self.d_count, cap,
                               self.donor_grid, self.donor_cell, self.s, self.status, stream)
        if self.fields is not None:
            B.overset_interp(self.ctx, self.donor_grid, self.donor_cell, self.s, self.d_count, cap, self.fields,
                             self.out, stream)

    def capture(self):
        """Capture one step as a HIP graph reading its poses from a fixed slot."""
        self.pose_slot = torch.zeros(self.ngrids * 12, dtype=torch.float64, device=self.dev)
        s = torch.cuda.Stream(self.dev)
        s.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(s):
            self.step(self.pose_slot)  # warm-up outside the graph
        torch.cuda.current_stream(self.dev).wait_stream(s)
        torch.cuda.synchronize(self.dev)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(self.pose_slot)
        self.graph = g

    def replay(self, poses_dev):
        self.pose_slot.copy_(poses_dev.reshape(-1), non_blocking=True)
        self.graph.replay()

    # ------------------------------------------------------------ results
    def results(self) -> dict:
        torch.cuda.synchronize(self.dev)
        n = int(self.d_count.item())
        m = min(n, self.capacity)
        cap = max(self.capacity, 1)
        r = {"count": n, "flags": self.flags.cpu().numpy(),
             "q_grid": self.q_grid[:m].cpu().numpy(), "q_node": self.q_node[:m].cpu().numpy(),
             "donor_grid": self.donor_grid[:m].cpu().numpy(), "donor_cell": self.donor_cell[:m].cpu().numpy(),
             "status": self.status[:m].cpu().numpy(),
             "s": self.s.reshape(3, cap)[:, :m].T.double().cpu().numpy(),
             "qx": self.qx.reshape(3, cap)[:, :m].T.double().cpu().numpy()}
        if self.fields is not None:
            r["values"] = self.out.reshape(4, cap)[:, :m].double().cpu().numpy()
        return r

"""Step drivers: device buffers for one overset system and the five C-ABI
calls of a time step (hole cut, fringe compaction, transform, donor search,
interpolation).

* `Assembly.step` runs a step on one stream (optionally replayed from a
  captured HIP graph).
* `Pipeline` runs consecutive steps on two streams with two buffer sets: the
  front half of step t+1 (hole cut + fringe compaction: bandwidth-bound,
  every CU busy) overlaps the back half of step t (transform, donor search,
  interpolation: latency-bound, few wavefronts). The library's scratch is
  split the same way (front-half scratch, back-half scratch), so each half
  only has to be ordered against itself; the donor search of step t+1 still
  follows that of step t on its stream, which keeps the warm start exact.

Grids are any objects with ``dims``, ``periodic``, ``X``, ``Y``, ``Z``
(FP64 body-frame coordinates, i fastest), ``blank_kind``, ``blank_prm`` and
``outer``; grid 0 is the stationary background.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


class StepBuffers:
    """Everything one step writes: flags, the query list, donors, values."""

    def __init__(self, dev, total: int, capacity: int, dtype):
        n = max(int(capacity), 1)
        self.capacity = int(capacity)
        self.flags = torch.empty(total, dtype=torch.uint8, device=dev)
        self.d_count = torch.zeros(1, dtype=torch.int64, device=dev)
        self.q_grid = torch.empty(n, dtype=torch.int32, device=dev)
        self.q_node = torch.empty(n, dtype=torch.int32, device=dev)
        self.qx = torch.empty(3 * n, dtype=dtype, device=dev)
        self.donor_grid = torch.empty(n, dtype=torch.int32, device=dev)
        self.donor_cell = torch.empty(n, dtype=torch.int32, device=dev)
        self.s = torch.empty(3 * n, dtype=dtype, device=dev)
        self.status = torch.empty(n, dtype=torch.int32, device=dev)
        self.out = torch.full((4 * n,), float("nan"), dtype=dtype, device=dev)


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
            mesh = getattr(g, "blank_mesh", None)
            gid = self.ctx.grid_add(g.dims, g.periodic, X, Y, Z, B.OV_BLANK_NONE if mesh is not None else g.blank_kind,
                                    tuple(g.blank_prm), tuple(g.outer))
            if mesh is not None:
                self.ctx.set_blank_mesh(gid, mesh)
        self.ctx.finalize()
        self.field_layout = 0
        self.frame_velocity = 0
        for k, v in (options or {}).items():
            self.set_option(k, v)
        self.ngrids = len(grids)
        self.total = self.ctx.total_nodes()
        self.node_off = np.array(self.ctx.node_offsets(), dtype=np.int64)
        self.fields = None
        if fields is not None:
            self.set_fields(fields)
        self.buf = StepBuffers(self.dev, self.total, 0, self.dtype)
        if capacity is not None:
            self.allocate(capacity)
        self.graph = None
        self.pose_slot = None

    def close(self):
        """Free the library context now (it holds device memory) instead of
        at interpreter exit."""
        self.graph = None
        if getattr(self, "ctx", None) is not None:
            self.ctx.close()

    def set_option(self, name: str, value: int):
        self.ctx.set_option(name, value)
        if name == "field_layout":
            self.field_layout = int(value)
        elif name == "frame_velocity":
            self.frame_velocity = int(value)

    # ------------------------------------------------------------ buffers
    def set_fields(self, fields):
        """fields: [4, total_nodes] (u, v, w, p). Stored as four blocks, or
        interleaved per node when the context's field layout is 1."""
        npdt = np.float32 if self.dtype == torch.float32 else np.float64
        f = np.asarray(fields).reshape(4, self.total)
        f = np.ascontiguousarray(f.T if self.field_layout == 1 else f, dtype=npdt)
        self.fields = torch.as_tensor(f).to(self.dev).reshape(-1).contiguous()

    def allocate(self, capacity: int):
        self.buf = StepBuffers(self.dev, self.total, capacity, self.dtype)

    def __getattr__(self, name):
        # flags, q_grid, ... of the single buffer set
        buf = self.__dict__.get("buf")
        if buf is not None and hasattr(buf, name):
            return getattr(buf, name)
        raise AttributeError(name)

    @property
    def capacity(self) -> int:
        return self.buf.capacity

    def count_queries(self, poses) -> int:
        """Hole cut + fringe compaction with capacity 0: returns the count."""
        p = self.as_poses(poses)
        b = self.buf
        B.overset_holecut(self.ctx, p, b.flags)
        B.overset_fringe_compact(self.ctx, self.nf, b.flags, None, None, 0, b.d_count)
        torch.cuda.synchronize(self.dev)
        self.ctx.status()  # clears the capacity bit this probe sets
        return int(b.d_count.item())

    def as_poses(self, poses):
        if isinstance(poses, torch.Tensor) and poses.is_cuda:
            return poses.reshape(-1)
        return torch.as_tensor(np.ascontiguousarray(poses, dtype=np.float64).reshape(-1)).to(self.dev)

    # ------------------------------------------------------------ the step
    def front(self, p, b: StepBuffers, stream=None):
        B.overset_holecut(self.ctx, p, b.flags, stream)
        B.overset_fringe_compact(self.ctx, self.nf, b.flags, b.q_grid, b.q_node, b.capacity, b.d_count, stream)

    def back(self, p, b: StepBuffers, stream=None):
        cap = b.capacity
        B.overset_transform(self.ctx, p, b.q_grid, b.q_node, b.d_count, cap, b.qx, stream)
        B.overset_donor_search(self.ctx, p, b.flags, b.q_grid, b.q_node, b.qx, b.d_count, cap, b.donor_grid,
                               b.donor_cell, b.s, b.status, stream)
        if self.fields is not None:
            B.overset_interp(self.ctx, b.donor_grid, b.donor_cell, b.s, b.d_count, cap, self.fields, b.out, stream)
            if self.frame_velocity:
                B.overset_frame_velocity(self.ctx, p, b.q_grid, b.donor_grid, b.d_count, cap, b.out, stream)

    # ------------------------------------------------------------ interpolation matrix
    def interp_matrix(self, b: StepBuffers | None = None, stream=None):
        """The step's interpolation matrix in ELL-8 form: (cols [capacity, 8]
        int32 global node indices, vals [capacity, 8] weights)."""
        b = self.buf if b is None else b
        cols = torch.empty((b.capacity, 8), dtype=torch.int32, device=self.dev)
        vals = torch.empty((b.capacity, 8), dtype=self.dtype, device=self.dev)
        B.overset_interp_matrix(self.ctx, b.donor_grid, b.donor_cell, b.s, b.d_count, b.capacity, cols, vals,
                                stream)
        return cols, vals

    def interp_apply(self, cols, vals, x, b: StepBuffers | None = None, y=None, layout: int = 0, stream=None):
        """y = M x. layout 0: x [nrhs, total_nodes], y [nrhs, capacity];
        layout 1 (interleaved per node): x [total_nodes, nrhs], y [capacity, nrhs]."""
        b = self.buf if b is None else b
        nrhs = x.shape[0] if layout == 0 else x.shape[1]
        if y is None:
            shape = (nrhs, b.capacity) if layout == 0 else (b.capacity, nrhs)
            y = torch.empty(shape, dtype=self.dtype, device=self.dev)
        B.overset_interp_apply(self.ctx, cols, vals, b.d_count, b.capacity, x, nrhs, y, layout, stream)
        return y

    def step(self, poses, stream=None):
        """One time step on one stream; nothing synchronises."""
        p = self.as_poses(poses)
        self.front(p, self.buf, stream)
        self.back(p, self.buf, stream)

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
    def results(self, b: StepBuffers | None = None) -> dict:
        b = self.buf if b is None else b
        torch.cuda.synchronize(self.dev)
        n = int(b.d_count.item())
        m = min(n, b.capacity)
        cap = max(b.capacity, 1)
        r = {"count": n, "flags": b.flags.cpu().numpy(),
             "q_grid": b.q_grid[:m].cpu().numpy(), "q_node": b.q_node[:m].cpu().numpy(),
             "donor_grid": b.donor_grid[:m].cpu().numpy(), "donor_cell": b.donor_cell[:m].cpu().numpy(),
             "status": b.status[:m].cpu().numpy(),
             "s": b.s.reshape(3, cap)[:, :m].T.double().cpu().numpy(),
             "qx": b.qx.reshape(3, cap)[:, :m].T.double().cpu().numpy()}
        if self.fields is not None:
            r["values"] = b.out.reshape(4, cap)[:, :m].double().cpu().numpy()
        return r


_EXECUTOR_STREAMS = {}


def executor_streams(dev, n: int):
    """The first n of the three streams that every Pipeline on device `dev`
    runs on, created together at the first call and kept for the process.
    The runtime multiplexes a process's streams onto a few hardware queues;
    streams that share one run their work one after another. torch's stream
    pool hands out a different set at every request, so the pipelines of one
    process would land on different queue mappings (some with two stages on
    one queue, which loses their overlap); shared streams give every pipeline
    the mapping of the first. Pipelines alive at the same time then order
    their stages among each other as well, which is still correct: every wait
    of the executor is for work submitted before it."""
    d = torch.device(dev)
    key = d.index if d.index is not None else torch.cuda.current_device()
    if key not in _EXECUTOR_STREAMS:
        _EXECUTOR_STREAMS[key] = [torch.cuda.Stream(d) for _ in range(3)]
    return _EXECUTOR_STREAMS[key][:n]


class Pipeline:
    """Pipelined execution of consecutive steps of an Assembly.
    stages=1: one stream and one buffer set (native only); stages=2: two
    streams (front = hole cut + fringe + compaction, back = transform +
    search + interpolation) and two buffer sets; stages=3: three streams
    (hole cut | fringe + compaction | back half) and three buffer sets
    (native only). native=True drives the library's C++ executor (ov_pipe_*:
    one host call per step); native=False issues the five calls from Python
    (optionally replaying per-half HIP graphs, see capture()). by_step (native,
    two or three streams): step t runs all its stages on stream t mod stages
    instead of stream g running stage group g of every step."""

    def __init__(self, asm: Assembly, capacity: int, native: bool = True, max_timed: int = 1024, stages: int = 2,
                 graphs: bool = False, threads: bool = False, by_step: bool = False):
        if stages not in (1, 2, 3) or (stages != 2 and not native):
            raise ValueError("stages must be 2, or 1 or 3 with the native executor")
        self.a = asm
        dev = asm.dev
        self.nsets = stages
        self.bufs = [StepBuffers(dev, asm.total, capacity, asm.dtype) for _ in range(stages)]
        self.streams = executor_streams(dev, stages)
        self.s_front = self.streams[0]
        self.s_back = self.streams[-1]
        self.native = None
        if native:
            self.native = B.NativePipe(asm.ctx, asm.nf, self.bufs, asm.fields, self.streams, max_timed)
            if graphs:
                self.native.use_graphs(True)
            if threads:
                self.native.set_threads(True)
            if by_step:
                self.native.set_by_step(True)
        self.by_step = bool(native and by_step)
        self.front_done = [torch.cuda.Event() for _ in range(2)]
        self.back_done = [torch.cuda.Event() for _ in range(2)]
        self.started = [False] * stages
        self.graphs = None
        cur = torch.cuda.current_stream(dev)
        for st in self.streams:
            st.wait_stream(cur)

    def wait_current(self):
        """Make every pipeline stream wait for the current stream."""
        cur = torch.cuda.current_stream(self.a.dev)
        for st in self.streams:
            st.wait_stream(cur)

    def submit(self, t: int, poses_dev, count_out=None, holecut_events=None):
        """Queue step t (poses on the device). Returns its buffer set.
        count_out: a 1-element device tensor that receives the step's query
        count; holecut_events: a pair of timing events around the hole cut."""
        k = t % self.nsets
        b = self.bufs[k]
        p = poses_dev.reshape(-1)
        if self.native is not None:
            self.native.submit(p, count_out)
            self.started[k] = True
            return b
        with torch.cuda.stream(self.s_front):
            if self.started[k]:
                self.s_front.wait_event(self.back_done[k])  # step t-2 no longer reads these buffers
            self._front(k, p, b, holecut_events)
            self.front_done[k].record(self.s_front)
        with torch.cuda.stream(self.s_back):
            self.s_back.wait_event(self.front_done[k])
            self._back(k, p, b)
            if count_out is not None:
                count_out.copy_(b.d_count, non_blocking=True)
            self.back_done[k].record(self.s_back)
        self.started[k] = True
        return b

    def submit_many(self, t0: int, poses_dev, counts_out=None):
        """Queue steps t0 .. t0 + n - 1 in one call of the native executor.
        poses_dev: [n, ngrids*12] device tensor; counts_out: int64[n] device tensor."""
        if self.native is None:
            raise RuntimeError("submit_many needs the native executor")
        self.native.submit_many(poses_dev, counts_out)
        for t in range(t0, t0 + int(poses_dev.shape[0])):
            self.started[t % self.nsets] = True

    def capture(self):
        """Capture, for each buffer set k, three single-stream HIP graphs: the
        hole cut, the fringe pass and the back half, all reading their poses
        from slot k. Afterwards submit() replays graphs instead of launching
        kernels one by one (the overlap between the two streams is kept:
        the graphs of different halves are launched on different streams)."""
        dev = self.a.dev
        self.slot = torch.zeros(2, self.a.ngrids * 12, dtype=torch.float64, device=dev)
        cap = torch.cuda.Stream(dev)
        cap.wait_stream(torch.cuda.current_stream(dev))
        self.graphs = []
        for k in range(2):
            b = self.bufs[k]
            p = self.slot[k]
            gs = []
            for part in ("holecut", "fringe", "back"):
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=cap):
                    if part == "holecut":
                        B.overset_holecut(self.a.ctx, p, b.flags, cap)
                    elif part == "fringe":
                        B.overset_fringe_compact(self.a.ctx, self.a.nf, b.flags, b.q_grid, b.q_node, b.capacity,
                                                 b.d_count, cap)
                    else:
                        self.a.back(p, b, cap)
                gs.append(g)
            self.graphs.append(gs)
        torch.cuda.synchronize(dev)

    def _front(self, k, p, b, holecut_events):
        if self.graphs is not None:
            self.slot[k].copy_(p, non_blocking=True)
        if holecut_events is not None:
            holecut_events[0].record(self.s_front)
        if self.graphs is not None:
            self.graphs[k][0].replay()
        else:
            B.overset_holecut(self.a.ctx, p, b.flags, self.s_front)
        if holecut_events is not None:
            holecut_events[1].record(self.s_front)
        if self.graphs is not None:
            self.graphs[k][1].replay()
        else:
            B.overset_fringe_compact(self.a.ctx, self.a.nf, b.flags, b.q_grid, b.q_node, b.capacity, b.d_count,
                                     self.s_front)

    def _back(self, k, p, b):
        if self.graphs is not None:
            self.graphs[k][2].replay()
        else:
            self.a.back(p, b, self.s_back)

    def join(self, stream=None):
        """Make `stream` (default: current) wait for everything submitted."""
        s = torch.cuda.current_stream(self.a.dev) if stream is None else stream
        if self.native is not None:
            self.native.join(s)
            return
        s.wait_stream(self.s_front)
        s.wait_stream(self.s_back)

    def back_stream(self, t: int):
        """The stream step t's back half runs on."""
        return self.streams[t % self.nsets] if self.by_step else self.streams[-1]

    def results(self, t: int) -> dict:
        self.join()
        return self.a.results(self.bufs[t % self.nsets])

    def close(self):
        """Wait for the executor's streams and free it."""
        if self.native is not None:
            self.native.close()
            self.native = None
        self.graphs = None

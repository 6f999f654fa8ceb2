"""overset_fringe_compact_noalloc (the fringe call for callers that cannot
allocate) against overset_fringe_compact, through the C ABI: the same flags,
query list and count, bit for bit, on two calls in a row whose second has a
smaller input (other grids, another context, the same static array); and a
context too large for the static array refused before any launch. Needs an
MI355X."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _both(w, t, precision):
    from paper_1910_09315_amd import binding as B
    from paper_1910_09315_amd.assembly import Assembly, StepBuffers
    a = Assembly(w.grids, w.nf, precision=precision)
    cap = 2 * a.count_queries(w.poses[t]) + 256
    a.allocate(cap)
    other = StepBuffers(a.dev, a.total, cap, a.dtype)
    p = a.as_poses(w.poses[t])
    B.overset_holecut(a.ctx, p, a.flags)
    other.flags.copy_(a.flags)
    B.overset_fringe_compact(a.ctx, w.nf, a.flags, a.q_grid, a.q_node, cap, a.d_count)
    B.overset_fringe_compact_noalloc(a.ctx, w.nf, other.flags, other.q_grid, other.q_node, cap, other.d_count)
    torch.cuda.synchronize()
    n = int(a.d_count.item())
    assert int(other.d_count.item()) == n and n > 0
    assert torch.equal(a.flags, other.flags)
    assert torch.equal(a.q_grid[:n], other.q_grid[:n]) and torch.equal(a.q_node[:n], other.q_node[:n])
    assert a.ctx.status() == 0
    a.close()
    return n


def test_noalloc_fringe_call_equals_the_allocating_call():
    # first the larger input, then a smaller one on the same static array
    n1 = _both(W.c4_small(steps=2), 1, "mixed")
    n2 = _both(W.c0(), 0, "fp64")
    n3 = _both(W.c1_small(steps=2), 1, "fp64")
    print("queries", n1, n2, n3, flush=True)
    assert n2 < n1


def test_noalloc_refuses_a_context_beyond_the_static_array():
    from paper_1910_09315_amd import binding as B
    from paper_1910_09315_amd.assembly import Assembly
    # a 2 x 2 x N background: one 64x8x8 tile per 32 nodes, so that the
    # tiles' scratch outgrows the array with a few million nodes
    nk = 8 * 330_000
    g = W.cartesian_grid((2, 2, nk), hi=(1.0, 1.0, 1000.0))
    a = Assembly([g], 0, precision="fp64")
    flags = torch.zeros(a.total, dtype=torch.uint8, device=a.dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=a.dev)
    with pytest.raises(B.OversetError, match="more than the static"):
        B.overset_fringe_compact_noalloc(a.ctx, 0, flags, None, None, 0, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    a.close()

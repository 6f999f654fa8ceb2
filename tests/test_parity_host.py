"""Host checks of the GPU parity gate itself (tests/parity.py), CPU only: a
result that differs from the oracle in a way the bar forbids must fail it.
The 'GPU' side here is the oracle's own result with one planted change."""
import numpy as np
import pytest

import oracle
import test_oracle_priority as P
from parity import compare


def _ref_and_gpu():
    b0 = 5 + 11 * (5 + 11 * 5)
    n1 = P.nearest_nodes(1, P.POSES[2, 9:], 1)[0]
    queries = [(0, b0, 2), (1, n1, oracle.CAUSE_BOUNDARY)]
    o = oracle.Oracle(P.GRIDS, nf=0)
    flags = np.zeros(o.total_nodes, np.uint8)
    for g, m, cause in queries:
        flags[P.OFF[g] + m] = oracle.ST_FRINGE | (cause << 2)
    qg = np.array([q[0] for q in queries], np.int32)
    qn = np.array([q[1] for q in queries], np.int32)
    d = o.donor_search(P.POSES, flags, qg, qn)
    ref = {"flags": flags, "q_grid": qg, "q_node": qn, **d}
    qx = np.stack([P.world(g, m) - P.POSES[g, 9:] for g, m, _ in queries])
    gpu = {"flags": flags.copy(), "count": len(qg), "q_grid": qg.copy(), "q_node": qn.copy(), "qx": qx,
           "donor_grid": d["donor_grid"].copy(), "donor_cell": d["donor_cell"].copy(), "s": d["s"].copy()}
    return o, ref, gpu


def test_identical_result_passes():
    o, ref, gpu = _ref_and_gpu()
    st = compare(o, P.POSES, ref, gpu, value_rtol=1.0, gate=2.0)
    assert st["near"] == 2 and st["near_other_cell"] == 0


@pytest.mark.parametrize("gate", [1e-3, 2.0])
def test_valid_donor_in_a_lower_priority_grid_fails(gate):
    """Query 0 (a background node cut by grid 2, inside grids 1 and 2) given
    its valid containing cell in grid 1: gated, it fails the bit-exact check;
    ungated (gate above every margin), it fails the donor-grid check, since
    the point is far from grid 2's outer boundary."""
    o, ref, gpu = _ref_and_gpu()
    x = P.world(0, int(ref["q_node"][0]))
    cell1 = P.closed_form(1, x)[0]
    gpu["donor_grid"][0] = 1
    gpu["donor_cell"][0] = cell1
    with pytest.raises(AssertionError):
        compare(o, P.POSES, ref, gpu, value_rtol=1.0, gate=gate)


def test_changed_flag_or_orphan_fails():
    o, ref, gpu = _ref_and_gpu()
    gpu["flags"][3] ^= 1
    with pytest.raises(AssertionError):
        compare(o, P.POSES, ref, gpu, value_rtol=1.0)
    o, ref, gpu = _ref_and_gpu()
    gpu["donor_grid"][1] = -1
    gpu["donor_cell"][1] = -1
    with pytest.raises(AssertionError):
        compare(o, P.POSES, ref, gpu, value_rtol=1.0)

"""Host logic of bench.py (CPU only): the refusal of more than one GPU, the
oracle comparison reported beside the bench line, and the rule that
recorded HBM traffic is dropped once the kernel sources differ from those
it was measured on."""
import json
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _step(n=6, seed=0):
    rng = np.random.default_rng(seed)
    return {"count": n, "flags": rng.integers(0, 4, 50).astype(np.uint8),
            "q_grid": np.zeros(n, np.int32), "q_node": np.arange(n, dtype=np.int32),
            "donor_grid": np.array([1, 1, -1, 1, 1, 1], np.int32)[:n],
            "donor_cell": np.arange(10, 10 + n, dtype=np.int32),
            "values": rng.standard_normal((4, n))}


def test_error_norms_of_identical_steps():
    ref = _step()
    e = bench.error_norms(ref, {k: (v.copy() if hasattr(v, "copy") else v) for k, v in ref.items()}, 3)
    assert e["flags_identical"] and e["queries_identical"] and e["orphans_identical"]
    assert e["donors_identical_frac"] == 1.0
    assert e["value_err_max_rel"] == 0.0 and e["value_err_rms_rel"] == 0.0


def test_error_norms_see_a_changed_donor_flag_and_value():
    ref = _step()
    gpu = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in ref.items()}
    gpu["flags"][7] ^= 1
    gpu["donor_cell"][0] += 1                  # one of five found donors differs
    gpu["values"][2, 3] += 1e-3 * np.abs(ref["values"][2]).max()
    e = bench.error_norms(ref, gpu, 0)
    assert not e["flags_identical"] and e["queries_identical"]
    assert e["donors_identical_frac"] == 0.8
    # values are compared over the queries with the same donor only
    assert abs(e["value_err_max_rel"] - 1e-3) < 1e-9


def test_error_norms_stop_at_a_different_query_list():
    ref = _step()
    gpu = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in ref.items()}
    gpu["q_node"][4] += 1
    e = bench.error_norms(ref, gpu, 0)
    assert not e["queries_identical"] and "donors_identical_frac" not in e


def test_recorded_traffic_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// version 1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = {"k_back|C9|fp64": {"bytes_per_launch": 1234, "sources": ["kernel.hip"],
                              "source_sha256": bench.source_hash(["kernel.hip"])}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic("k_back|C9|fp64") == 1234
    assert bench.recorded_traffic("k_back|C9|mixed") is None
    src.write_text("// version 2\n")
    assert bench.recorded_traffic("k_back|C9|fp64") is None

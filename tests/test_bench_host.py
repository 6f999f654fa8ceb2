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


def test_driver_argument_set_times_the_back_half():
    """The driver runs `--gpus 1 --steps 20 --warmup 5`: the executor must
    time k_back on several of those steps (counted from the first timed
    step, not from the executor's first step)."""
    args = bench.make_parser().parse_args(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert args.roofline == "back" and args.time_every > 0
    got = bench.sampled_steps(args.steps, args.time_every)
    assert got[0] == 0 and len(got) >= 3 and max(got) < args.steps


def test_counter_runs_are_detected(monkeypatch):
    monkeypatch.delenv("ROCPROF_COUNTER_COLLECTION", raising=False)
    assert not bench.profiler_counting()
    for v in ("1", "True", "true"):
        monkeypatch.setenv("ROCPROF_COUNTER_COLLECTION", v)
        assert bench.profiler_counting()
    monkeypatch.setenv("ROCPROF_COUNTER_COLLECTION", "0")
    assert not bench.profiler_counting()


def test_roofline_objects_from_work_counters():
    """Per-launch algorithmic work from summed counters, and the bound set by
    the larger fraction."""
    stat = [0] * 9
    stat[bench.ST_BACK] = 2
    stat[bench.ST_CELLS] = 2 * 1000
    stat[bench.ST_ITERS] = 2 * 3000
    r = bench.back_roofline(stat, 500.0, 10e-6, "fp64", 8, 800, None)
    hb = r["hbm_view"]["algorithmic_bytes_per_launch"]
    assert hb == bench.back_bytes_per_query(8) * 500 + bench.BACK_BYTES_PER_CELL * 1000 + 32 * 800
    fl = r["alu_view"]["algorithmic_flops_per_launch"]
    assert fl == bench.FLOPS_PER_CELL["fp64"] * 1000 + bench.FLOPS_PER_NEWTON_ITER * 3000 + bench.FLOPS_PER_QUERY * 500
    assert r["bound"] == ("hbm" if r["hbm_view"]["frac"] >= r["alu_view"]["frac"] else "alu")
    stat = [0] * 9
    stat[bench.ST_HC_CALLS] = 4
    stat[bench.ST_FLAG_W] = 4 * 4096
    stat[bench.ST_BASE_R] = 4 * 1024
    stat[bench.ST_HC_NODES] = 4 * 100
    h = bench.holecut_roofline(stat, 5e-6, "mixed", 10, "t")
    assert h["algorithmic_bytes_per_launch"] == 4096 + 1024 + 13 * 100 + 32 * 10

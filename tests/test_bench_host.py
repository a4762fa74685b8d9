"""Host-side parts of bench.py (no GPU): the one-GPU guard and the oracle leg
whose results the bench compares the timed run with."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_returns_the_oracle_reference_on_a_full_run():
    import bench
    from paper_2503_01276_amd import workloads as W

    info, ref = bench.cpu_baseline("t3", 4)
    cfg = W.PRESETS["t3"]
    M = cfg.n_cont * (1 + cfg.dim)
    assert info["kind"] == "oracle" and info["cores"] == 4 and info["value"] > 0
    assert ref["A"].shape == (cfg.n_points, M, M)
    g = np.asarray(ref["g"])
    assert g.size == cfg.n_fine ** cfg.dim and np.all(np.isfinite(g)) and np.abs(g).max() > 0


def test_cpu_baseline_sample_has_no_reference():
    import bench

    info, ref = bench.cpu_baseline("t3d", 4)  # 3D: a bounded forward-only sample
    assert ref is None and "sample" in info and info["value"] > 0

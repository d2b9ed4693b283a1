"""Host-side checks of bench.py's contract (no GPU needed)."""
from __future__ import annotations

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_exits_with_message():
    """The build measures one GPU; --gpus N > 1 must stop with a message
    (before touching a device)."""
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_workload_recipes():
    """The benchmark workload and the p-sweep points: element counts,
    degrees and the stretching that gives aspect ratio 8."""
    wl = bench.workload("c2a")
    assert wl["n"] == (16, 16, 16) and wl["p"] == 8
    assert abs(wl["alpha"] ** 15 - 8.0) < 1e-12
    wl = bench.workload("c2b")
    assert wl["n"] == (8, 8, 8) and wl["p"] == 16
    assert abs(wl["alpha"] ** 7 - 8.0) < 1e-12
    for p in bench.SWEEP:
        w = bench.workload(f"c3p{p}")
        assert w["p"] == p and w["n"][0] == int(round(215.44 / p)) and bench.is_uniform(w)


def test_smoother_flop_count():
    """37 n_S^3 flop per star (Alg. 1 count), corners excluded: 0.612 GFLOP
    at 16^3, p = 8."""
    fl = bench.smoother_flops((16, 16, 16), 8)
    assert fl == 37.0 * 15 ** 3 * (17 ** 3 - 8)
    assert abs(fl - 0.612e9) < 0.001e9


def test_smoother_kernel_names():
    assert bench.smoother_kernel(2, "float") == "k_smoother_small<float, 3>"
    assert bench.smoother_kernel(4, "double") == "k_smoother_small<double, 8>"
    assert bench.smoother_kernel(8, "float") == "k_smoother_mfma<float, 1>"


def test_coarse_level_policy():
    """Degree-1 levels below p_0: six at p <= 4; one at 4 < p <= 8 on uniform
    meshes of at least 16^3 elements; none otherwise (stretched meshes,
    small meshes, p >= 12)."""
    assert bench.coarse_levels(2, True, 8) == 6 and bench.coarse_levels(4, False, 4096) == 6
    assert bench.coarse_levels(8, True, 16 ** 3) == 1 and bench.coarse_levels(8, True, 40 ** 3) == 1
    assert bench.coarse_levels(8, True, 8 ** 3) == 0 and bench.coarse_levels(12, True, 40 ** 3) == 0
    wl = bench.workload("c2a")
    assert not bench.is_uniform(wl) and bench.coarse_levels(8, bench.is_uniform(wl), 16 ** 3) == 0
    wl = bench.workload("c4")
    assert bench.is_uniform(wl) and bench.coarse_levels(8, True, 32 ** 3) == 1


def test_headline_workload_and_counts():
    """The headline is the 32^3, p = 8 mixed-precision configuration (16.8M
    unknowns); operator count 73 (p-1)^3 + 24 p^3 per element; unique
    condensed unknowns (np-1)^3 - n_e (p-1)^3 (5,341,951 at 32^3, p = 8)."""
    wl = bench.workload("c4")
    assert wl["n"] == (32, 32, 32) and wl["p"] == 8 and wl["lam"] == 0.0
    assert wl["lengths"] == (1.0, 0.5, 1.0)
    assert bench.n_hat(wl["n"], 8) == 5341951
    assert bench.op_flops((1, 1, 1), 8) == 73 * 343 + 24 * 512
    r = bench.roofline(1e9, 1e9, 1e-3, "f64")      # intensity 1 < ridge: HBM-bound
    assert r["bound"] == "hbm" and abs(r["achieved"] - 1000.0) < 1e-9
    r = bench.roofline(1e12, 1e9, 1e-1, "f32")     # intensity 1000: ALU-bound
    assert r["bound"] == "mfma" and abs(r["frac"] - 10.0 / 157.3) < 1e-12

"""Host logic of bench.py, on the CPU: the one-GPU guard, the classification of
true residuals against the stopping threshold in force, and the use of the committed
HBM counter summary only for the kernel source, kernel and launch shape it was taken
with."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def _st(r0, b, true_rel):
    return {"rnorm0": r0, "bnorm": b, "true_rel_res": true_rel}


def test_residual_gate_splits_tol_and_floor_bound_solves():
    tol = 1e-10
    stats = [
        _st(1.0, 1.0, 0.5e-10),     # tol-bound: true = 0.5 tol r0
        _st(1.0, 10.0, 2.0e-10),    # tol-bound (1e-10 > 1e-13): 2 tol r0
        _st(1e-6, 1.0, 1e-7),       # floor-bound (1e-16 < 1e-14): true = 1e-13 = 10 floor
        _st(0.0, 1.0, 0.0),         # zero residual: floor-bound, true 0
    ]
    g = bench._residual_gate(stats, tol)
    assert g["solves"] == 4 and g["floor_bound_solves"] == 2
    assert g["tol_bound_max_true_over_tol_r0"] == pytest.approx(2.0)
    assert g["floor_bound_max_true_over_floor_b"] == pytest.approx(10.0)
    assert g["max_true_rel_res"] == pytest.approx(1e-7)


def test_measured_traffic_only_for_the_counted_source_and_shape(monkeypatch):
    prof = os.path.join(ROOT, "profiles", "fld_lognormal_L6-9_fp64_hbm_counters.txt")
    kv = dict(line.split(": ", 1) for line in open(prof).read().splitlines() if line.startswith("traffic_"))
    kernel, blocks = kv["traffic_kernel"], int(kv["traffic_max_blocks"])
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: kv["traffic_source_sha256_prefix"])
    assert bench._measured_traffic(kernel, blocks) == pytest.approx(float(kv["traffic_kib_per_dispatch"]) * 1024)
    assert bench._measured_traffic(kernel, blocks * 2) is None
    assert bench._measured_traffic("k_pass_b<double>", blocks) is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 16)
    assert bench._measured_traffic(kernel, blocks) is None


def test_algorithmic_bytes_per_slot():
    # pass A: r, p_old, d, three coefficients, 3 B of neighbour table; writes p, q
    assert bench.PASS_A_BYTES == 67
    # pass B: x, r, p, q, d; writes x, r
    assert bench.PASS_B_BYTES == 56

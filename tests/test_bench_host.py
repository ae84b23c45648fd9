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
    assert bench._measured_traffic("k_other<double>", blocks) is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 16)
    assert bench._measured_traffic(kernel, blocks) is None


def test_algorithmic_bytes_per_slot():
    # the method's bytes per cell and CG iteration, the figures the rooflines quote:
    # FP64: the operator sweep of Jacobi PCG 69 + its update sweep 56; FP32 inner 37 + 28
    assert bench.ALG_BYTES_FP64 == 125 and bench.ALG_BYTES_FP32 == 65
    # the fused sweep moves p, s, w, x, r, rs, three coefficients and 3 B of neighbour
    # table, and writes p, s, x, r, w
    assert bench.SWEEP_BYTES == 115 and bench.SWEEP_BYTES_FORMED == 100 and bench.SWEEP_BYTES_FP32 == 59


def test_roofline_of_timed_sweeps():
    stats = [{"sweep_ms": 2.0, "n_timed": 4, "n_leaf": 1_000_000},
             {"sweep_ms": 1.0, "n_timed": 2, "n_leaf": 1_000_000}]
    r = bench._roofline(stats, 125, "k", "n")
    # 6 launches over 1e6 cells at 125 B in 3 ms
    assert r["achieved"] == pytest.approx(6 * 125e6 / 3e-3 / 1e9, rel=1e-6)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["timed_launches"] == 6 and r["avg_launch_us"] == pytest.approx(500.0)
    assert bench._roofline([{"sweep_ms": 0.0, "n_timed": 0, "n_leaf": 1}], 125, "k", "n") is None


def test_schedule_is_fine_first_with_restrictions():
    class H:
        base_level, max_level = 6, 8

    class P:
        hierarchy, dt_coarse = H, 1.0

    ops = bench._schedule(P)
    solves = [(l, dt) for k, l, dt in ops if k == "solve"]
    assert solves == [(8, 0.25), (8, 0.25), (7, 0.5), (8, 0.25), (8, 0.25), (7, 0.5), (6, 1.0)]
    assert [l for k, l, _ in ops if k == "restrict"] == [8, 8, 7]

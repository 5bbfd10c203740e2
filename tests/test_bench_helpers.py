"""The benchmark's reporting arithmetic (CPU only): which roofline a kernel is reported
against, when the committed HBM counter summary applies, and the hot-path byte count."""

import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_roofline_bound_follows_the_machine_balance():
    # FP64: 9.8 flop/B balance (78.6 TFLOP/s over 8 TB/s)
    alu = bench.update_roofline(10.0, 1e9, 11e9, 1, "none", "fp64")
    assert alu["bound"] == "alu" and alu["unit"] == "TFLOP/s" and alu["peak"] == bench.FP64_PEAK_TFS
    assert alu["achieved"] == pytest.approx(1.1) and alu["frac"] == pytest.approx(1.1 / bench.FP64_PEAK_TFS)
    hbm = bench.update_roofline(10.0, 1e9, 5e9, 1, "none", "fp64")
    assert hbm["bound"] == "hbm" and hbm["unit"] == "GB/s" and hbm["achieved"] == pytest.approx(100.0)
    # FP32 storage: against the FP32 peak, so the same intensity is below its balance
    f32 = bench.update_roofline(10.0, 1e9, 11e9, 1, "none", "fp32")
    assert f32["bound"] == "hbm"
    # per-launch averages
    two = bench.update_roofline(10.0, 2e9, 30e9, 2, "none", "fp64")
    assert two["avg_launch_ms"] == 5.0 and two["bytes_per_launch"] == 1e9


def test_measured_traffic_applies_only_to_its_configuration():
    path = os.path.join(ROOT, "profiles", "k_flush_diamond_traffic.json")
    with open(path) as f:
        rec = json.load(f)
    got = bench.measured_traffic("diamond", rec["workload"], "fp64")
    if rec["kernel_sources_sha1"] == bench.update_kernel_digest():
        assert got == rec["hbm_bytes_per_launch"]
        # FP64 counters are not the FP32 kernel's, nor another configuration's
        assert bench.measured_traffic("diamond", rec["workload"], "fp32") is None
        assert bench.measured_traffic("diamond", rec["workload"] + ", window 8", "fp64") is None
    else:
        assert got is None  # the kernel changed since the counters were taken
    assert bench.measured_traffic("no_such_workload", None, "fp64") is None


def test_hot_path_bytes():
    """The modelled hot path is labelled a model, carries no roofline bound of its own, and counts
    the update's bytes, 8 vectors per seed iteration and the matrix once per sweep."""
    h = bench.hot_path(1e9, 10, 1000, 2.0, matrix_bytes=12e3, sweeps=10)
    assert h["bytes"] == 1e9 + 10 * 8 * 16 * 1000 + 12e3 * 10
    assert h["achieved_gbs"] == pytest.approx(h["bytes"] / 1e9 / 2.0)
    assert "bound" not in h and "model" in h


def test_measured_hot_path_applies_only_to_current_sources_and_workload():
    path = os.path.join(ROOT, "profiles", "hot_path_diamond_traffic.json")
    if not os.path.exists(path):
        assert bench.measured_hot_path("diamond", "anything") is None
        return
    with open(path) as f:
        rec = json.load(f)
    got = bench.measured_hot_path("diamond", rec["workload"])
    if rec["library_sources_sha1"] == bench.library_digest():
        assert got is not None and got["hbm_bytes_per_step"] == rec["hbm_bytes_per_step"]
        assert bench.measured_hot_path("diamond", rec["workload"] + ", other") is None
    else:
        assert got is None


def test_measured_kernels_apply_only_to_current_sources_and_workload():
    """The per-kernel record (trace durations with counter bytes) is reported only while both
    committed summaries were taken on the current library sources and this workload."""
    paths = [os.path.join(ROOT, "profiles", n) for n in ("kernels_diamond_stats.json", "hot_path_diamond_traffic.json")]
    if not all(os.path.exists(p) for p in paths):
        assert bench.measured_kernels("diamond", "anything") is None
        return
    recs = []
    for p in paths:
        with open(p) as f:
            recs.append(json.load(f))
    got = bench.measured_kernels("diamond", recs[0]["workload"])
    if all(r["library_sources_sha1"] == bench.library_digest() for r in recs) and recs[0]["workload"] == recs[1]["workload"]:
        assert got and any("k_spmv" in k["kernel"] for k in got)
        for k in got:
            assert k["achieved_gbs"] == pytest.approx(k["memory_side_bytes_per_launch"] / 1e3 / k["avg_us"])
        assert bench.measured_kernels("diamond", recs[0]["workload"] + ", other") is None
    else:
        assert got is None


def test_more_than_one_gpu_is_refused_with_a_message():
    import subprocess

    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""

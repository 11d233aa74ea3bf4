"""Host-side logic of bench.py (no GPU): the single-GPU refusal, the algorithmic byte and
operation counts the rooflines divide by, the roofline arithmetic, the HBM-traffic summary
built from rocprofv3 counter files, and the rule that a traffic summary is used only while
the step kernel's sources are the ones it was taken on."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_first_order_bytes_are_itemised():
    N, F, K = 1000, 7840, 80
    # intensities read and written, faces (cell pair + A n + A w.n), CSR, FP64 cell state
    assert bench.algorithmic_bytes(N, F, K, "f32") == N * K * 8 + F * (8 + 16) + (N + 1) * 4 + 2 * F * 4 + 120 * N
    assert bench.algorithmic_bytes(N, F, K, "f64") == N * K * 16 + F * (8 + 32) + (N + 1) * 4 + 2 * F * 4 + 120 * N


def test_plm_bytes_are_about_five_first_order_steps():
    # at the PLM workload's shape (7.84 faces per cell, 80 angles)
    N, K = 262144, 80
    F = int(7.84 * N)
    for dtype, lo, hi in (("f32", 4.8, 5.1), ("f64", 5.2, 5.5)):
        first = bench.algorithmic_bytes(N, F, K, dtype)
        plm = bench.plm_algorithmic_bytes(N, F, K, dtype)
        assert lo < plm / first < hi, (dtype, plm / first)
        s = 4 if dtype == "f32" else 8
        # two first-order steps, 8 more intensity-sized passes, the gradient's face weights and
        # the reconstruction offsets
        assert plm == 2 * first + 8 * N * K * s + F * (8 + 6 * s) + F * 6 * s


def test_operation_count():
    N, F, K = 10, 40, 8
    assert bench.algorithmic_ops(N, F, K) == N * K * bench.SOURCE_OPS_PER_CA + F * K * bench.FACE_OPS_PER_FA


def test_roofline_arithmetic():
    r = bench._roofline(2.0, 8e9)  # 8 GB in 2 ms = 4 TB/s
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0) and r["frac"] == pytest.approx(0.5)
    r = bench._roofline(1.0, 1e9, ops=bench.ALU_PEAK_TOPS * 1e9 / 2)
    assert r["other"]["bound"] == "alu" and r["other"]["frac"] == pytest.approx(0.5, rel=1e-3)


def _counter_file(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_counter_summary_scales_by_the_copy_kernel(tmp_path):
    """FETCH_SIZE reads half of the copy's known bytes here (scale 2) and WRITE_SIZE all of them
    (scale 1); counter values are KiB per dispatch."""
    copy_bytes = 1024 * 1024 * 100
    (tmp_path / "fetch").mkdir()
    (tmp_path / "write").mkdir()
    _counter_file(tmp_path / "fetch" / "f_counter_collection.csv", [
        {"Kernel_Name": "void at::native::neg_kernel", "Counter_Name": "FETCH_SIZE", "Counter_Value": copy_bytes / 2 / 1024},
        {"Kernel_Name": "void k_step<float, 8, 10, 1, true, 2>(rt_step_args, long)", "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 1000.0},
        {"Kernel_Name": "void k_step<float, 8, 10, 1, true, 2>(rt_step_args, long)", "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 3000.0},
        {"Kernel_Name": "void k_step<double, 8, 10, 1, true, 2>(rt_step_args, long)", "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 5000.0},
    ])
    _counter_file(tmp_path / "write" / "w_counter_collection.csv", [
        {"Kernel_Name": "void at::native::neg_kernel", "Counter_Name": "WRITE_SIZE", "Counter_Value": copy_bytes / 1024},
        {"Kernel_Name": "void k_step<float, 8, 10, 1, true, 2>(rt_step_args, long)", "Counter_Name": "WRITE_SIZE",
         "Counter_Value": 500.0},
        {"Kernel_Name": "void k_step<double, 8, 10, 1, true, 2>(rt_step_args, long)", "Counter_Value": 700.0,
         "Counter_Name": "WRITE_SIZE"},
    ])
    s = bench.counters_summary(str(tmp_path), copy_bytes)
    assert s["scale"]["FETCH_SIZE"] == pytest.approx(2.0) and s["scale"]["WRITE_SIZE"] == pytest.approx(1.0)
    f32 = s["kernels"]["step_upwind1_f32"]
    assert f32["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2)  # mean of the two launches, scaled
    assert f32["write_bytes_per_launch"] == pytest.approx(500.0 * 1024)
    assert f32["hbm_bytes_per_launch"] == pytest.approx((4000.0 + 500.0) * 1024) and f32["launches"] == 2
    assert s["kernels"]["step_upwind1_f64"]["hbm_bytes_per_launch"] == pytest.approx((10000.0 + 700.0) * 1024)
    assert s["source_hash"] == bench.kernel_source_hash()


def test_traffic_is_used_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    summary = {"source_hash": "0123456789abcdef", "kernels": {"step_upwind1_f32": {"hbm_bytes_per_launch": 42.0}}}
    (prof / "traffic.json").write_text(json.dumps(summary))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0123456789abcdef")
    assert bench.measured_traffic("step_upwind1_f32") == 42.0
    assert bench.measured_traffic("step_upwind1_f64") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "fedcba9876543210")
    assert bench.measured_traffic("step_upwind1_f32") is None


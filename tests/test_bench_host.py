"""CPU tests of the measurement harness (bench.py): the rocprofv3 summary
writers scale the counters by the calibration kernel and classify the
dispatches as documented, a stale summary gives no traffic figure, the
committed summaries match the kernel sources they name, and a request for
more than one GPU is refused (this build measures one GPU)."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "t_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_traffic_summary_scaling_and_classes(tmp_path):
    calib_kib = bench.CALIB_ELEMS * 8 / 1024.0
    fetch = [("at::native::vectorized_elementwise_kernel<neg>", "FETCH_SIZE", calib_kib / 2)] * 3 + [
        ("k_sweep<double, true, 6, 1, double, double>", "FETCH_SIZE", 100.0),
        ("k_sweep<double, true, 6, 1, double, double>", "FETCH_SIZE", 300.0),
        ("k_sweep<double, false, 6, 2, double, double>", "FETCH_SIZE", 50.0),
        ("k_spmv<0, 8>", "FETCH_SIZE", 1000.0)]
    write = [("at::native::vectorized_elementwise_kernel<neg>", "WRITE_SIZE", calib_kib)] * 3 + [
        ("k_sweep<double, true, 6, 1, double, double>", "WRITE_SIZE", 10.0),
        ("k_sweep<double, true, 6, 1, double, double>", "WRITE_SIZE", 30.0),
        ("k_sweep<double, false, 6, 2, double, double>", "WRITE_SIZE", 5.0),
        ("k_spmv<0, 8>", "WRITE_SIZE", 100.0)]
    _write_counters(tmp_path / "f", fetch)
    _write_counters(tmp_path / "w", write)
    out = tmp_path / "summary.md"
    bench.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), "cmd f", "cmd w", out_file=str(out),
                          label="test")
    text = out.read_text()
    assert f"source-hash: {bench.source_hash()}" in text
    assert "scale: FETCH x2.0000, WRITE x1.0000" in text
    # forward sweep: mean fetch 200 KiB read at half rate -> 400 KiB, plus 20 KiB written
    assert f"traffic-bytes-per-launch k_sweep(forward) {1024 * (400 + 20):.0f}" in text
    assert f"traffic-bytes-per-launch k_sweep(backward) {1024 * (100 + 5):.0f}" in text
    assert f"traffic-bytes-per-launch k_spmv {1024 * (2000 + 100):.0f}" in text
    assert bench.traffic_for("k_sweep(forward)", str(out)) == pytest.approx(1024 * 420)
    # a summary of other sources gives no figure
    out.write_text(text.replace(bench.source_hash(), "0" * 16))
    assert bench.traffic_for("k_sweep(forward)", str(out)) is None


def test_tcc_summary_hit_rate(tmp_path):
    _write_counters(tmp_path / "c", [
        ("k_sweep<double, true, 6, 1, double, double>", "TCC_HIT_sum", 30.0),
        ("k_sweep<double, true, 6, 1, double, double>", "TCC_MISS_sum", 70.0),
        ("k_spmv<0, 8>", "TCC_HIT_sum", 50.0),
        ("k_spmv<0, 8>", "TCC_MISS_sum", 50.0)])
    out = tmp_path / "l2.md"
    bench.tcc_summary(str(tmp_path / "c"), "cmd", str(out), "test")
    text = out.read_text()
    assert "| k_sweep(forward) | 1 | 30 | 70 | 0.300 |" in text
    assert "| k_spmv | 1 | 50 | 50 | 0.500 |" in text


def test_committed_profiles_match_sources():
    """Every committed summary names the kernel sources it was taken from;
    the traffic figure the benchmark reports is only used while they match."""
    prof = os.path.join(ROOT, "profiles")
    names = [f for f in os.listdir(prof) if f.endswith(".md")]
    assert names
    for f in names:
        with open(os.path.join(prof, f)) as fh:
            text = fh.read()
        assert "rocprofv3" in text, f
        assert f"source-hash: {bench.source_hash()}" in text, f
    assert bench.traffic_for("k_sweep(forward)") is not None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

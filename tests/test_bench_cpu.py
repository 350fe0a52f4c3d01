"""Host logic of the benchmark line (no GPU): the roofline picks the kernel
class with the most summed time and divides its algorithmic work by its
average launch duration; the factorization class takes the elimination flops
it is given; the HBM classes divide algorithmic bytes by time; the traffic
figure is read from the committed summary only while the sources it was taken
on are unchanged."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _prof():
    return {
        "gemm_solve": {"launches": 24, "ms": 15.0, "flops": 24 * 2.0e10, "bytes": 24 * 1.0e9},
        "gemm_factor": {"launches": 100, "ms": 12.0, "flops": 1.0e12, "bytes": 5.0e10},
        "gemm_krylov": {"launches": 10, "ms": 3.0, "flops": 1.0e11, "bytes": 1.0e10},
        "spmm": {"launches": 8, "ms": 1.0, "flops": 1.0e9, "bytes": 4.0e9},
        "solve_gather": {"launches": 24, "ms": 2.0, "flops": 0.0, "bytes": 1.2e10},
        "elemwise": {"launches": 5, "ms": 0.5, "flops": 0.0, "bytes": 0.0},
    }


def test_roofline_picks_dominant_class():
    r = bench.roofline(_prof(), 1)
    assert r["kernel"] == "gemm_solve" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    # 2e10 flops per launch over 0.625 ms per launch = 32 TFLOP/s
    assert r["avg_launch_us"] == pytest.approx(625.0)
    assert r["achieved"] == pytest.approx(32.0)
    assert r["frac"] == pytest.approx(32.0 / bench.PEAK_FP64_TFLOPS)
    assert r["flops_per_launch"] == pytest.approx(2.0e10)


def test_roofline_factor_uses_elimination_flops():
    # the method's work per query (elimination only) times the queries profiled
    r = bench.roofline(_prof(), 2, method_factor_flops=3.0e11, kernel="gemm_factor")
    assert r["kernel"] == "gemm_factor"
    assert r["achieved"] == pytest.approx(2 * 3.0e11 / 12.0e-3 / 1e12)
    assert "flops_note" in r


def test_roofline_fp32_peak():
    r = bench.roofline(_prof(), 1, fp32=True)
    assert r["peak"] == bench.PEAK_FP32_TFLOPS


def test_hbm_rates():
    s = bench.spmm_rate(_prof())
    assert s["bound"] == "hbm" and s["achieved"] == pytest.approx(4.0e9 / 1.0e-3 / 1e9)
    g = bench.spmm_rate(_prof(), "solve_gather")
    assert g["frac"] == pytest.approx(1.2e10 / 2.0e-3 / 1e9 / bench.PEAK_HBM_GBS)
    # a class without byte counts, or not profiled, has no rate
    assert bench.spmm_rate(_prof(), "elemwise") is None
    assert bench.spmm_rate({}, "spmm") is None
    assert bench.spmm_rate(None) is None


def test_traffic_only_for_unchanged_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text(f"# header\nsource_hash: {bench.gemm_source_hash()}\ngemm_solve_bytes_per_launch: 1.5e9\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("gemm_solve") == pytest.approx(1.5e9)
    assert bench.measured_traffic("gemm_factor") is None
    f.write_text("source_hash: 0000000000000000\ngemm_solve_bytes_per_launch: 1.5e9\n")
    assert bench.measured_traffic("gemm_solve") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("gemm_solve") is None

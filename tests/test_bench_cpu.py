"""Host logic of bench.py: the one-GPU guard, the roofline classification and
the lookup of measured HBM traffic (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_roofline_bound_follows_the_ridge_point():
    ridge = bench.FP32_PEAK_TFLOPS * 1e12 / (bench.HBM_PEAK_GBS * 1e9)
    assert ridge == pytest.approx(9.825, rel=1e-3)
    # 1 GB and 1 ms: 1000 GB/s; 5 GFLOP: intensity 5 < ridge, HBM-bound
    r, tfl = bench.roofline_of(1e9, 5e9, 1e-3, None)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(1000.0) and r["frac"] == pytest.approx(1000.0 / bench.HBM_PEAK_GBS, abs=5e-5)
    assert tfl == pytest.approx(5.0)
    # intensity 20 > ridge: ALU-bound, the achieved rate is the FP32 rate
    r, tfl = bench.roofline_of(1e9, 20e9, 1e-3, 123.0)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["traffic"] == 123.0
    assert r["achieved"] == pytest.approx(20.0) and r["frac"] == pytest.approx(20.0 / bench.FP32_PEAK_TFLOPS, abs=5e-5)


def test_two_step_pass_is_hbm_bound_by_intensity():
    # the two-step pass moves 28 B per node and does two updates' arithmetic
    flop = 2 * bench.FLOP_PER_LUP[True]
    assert flop / bench.BYTES_PER_LUP < bench.FP32_PEAK_TFLOPS * 1e12 / (bench.HBM_PEAK_GBS * 1e9)


def test_measured_traffic_matches_source_size_and_tile_height():
    from paper_1902_02999_amd.profiling import kernel_sha
    for key, files in bench.TRAFFIC_FILES.items():
        for path in ([files] if isinstance(files, str) else files):
            if not os.path.exists(path):
                continue
            with open(path) as f:
                t = json.load(f)
            src = os.path.join(ROOT, "paper_1902_02999_amd", "csrc", t.get("kernel_source", "mlb_kernels.hip"))
            assert t["bytes_per_launch"] > 0 and t["nodes"] > 0
            # a different problem size never takes the figure
            assert bench.measured_traffic(t["nodes"] + 1, key, t.get("tile_rows")) is None
            if t.get("kernel_sha") != kernel_sha(src):
                continue   # taken on an older kernel source
            got = bench.measured_traffic(t["nodes"], key, t.get("tile_rows"))
            assert got is not None
            if t.get("tile_rows") is not None:
                # another tile height does not take this file's figure
                other = bench.measured_traffic(t["nodes"], key, t["tile_rows"] + 1000)
                assert other is None

"""bench.py's one-line JSON report, on the GPU: a short run of the default
workload at 512^2 must print exactly one JSON line with every field of the
report, a roofline object for the dominant kernel and the oracle's timing."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_default_report_fields():
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--n", "512", "--steps", "40", "--warmup", "4",
           "--no-autotune", "--tblock", "2", "--tile-rows", "17", "--cpu-seconds", "1"]
    print("running", " ".join(cmd[2:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["metric"] == "MLUPS" and d["unit"] == "MLUPS" and d["n_gpus"] == 1
    assert d["steps"] == 40 and d["warmup"] == 4 and d["higher_is_better"] is True
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert d["dtype"] == "f32" and d["data"] == "synthetic" and d["vs_baseline"] is None
    assert d["config"]["workload"] == "bump_channel_512x512" and d["config"]["nodes"] == 512 * 512
    assert d["config"]["tblock"] == 2 and d["config"]["tile_rows"] == 17
    # MLUPS and milliseconds per step describe the same timed region
    # (ms_per_step carries five decimals)
    assert d["value"] == pytest.approx(512 * 512 / (d["ms_per_step"] * 1e3), rel=1e-3 + 5e-6 / d["ms_per_step"])
    rf = d["roofline"]
    assert set(rf) == {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["achieved"] > 0 and rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], abs=1e-4)
    assert rf["traffic"] is None and d["config"]["traffic_GBps"] is None   # no counter summary at this size
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == "MLUPS" and cb["value"] > 0 and cb["cores"] >= 1
    assert "512x512" in cb["sample"]
    assert cb["value_1_thread"] > 0   # the oracle on one thread beside all cores
    # the roofline comes from the bulk two-step passes timed alone
    assert d["config"]["launch_us"] > 0
    # the other half of the metric: wall seconds to R <= 1e-6, warm against cold
    wc = d["config"]["warm_vs_cold"]
    assert wc["cold_s"] > 0 and wc["warm_s"] > 0 and wc["cold_steps_median"] > 0

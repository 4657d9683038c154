"""bench.py's JSON line on the GPU (a short headline run, in process)."""
import json
import sys

import pytest

from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


def test_headline_bench_line(monkeypatch, capsys):
    need_gpu()
    import bench
    say("bench --no-extras, 2 chunks of 64 steps, one case")
    monkeypatch.setattr(sys, "argv", ["bench.py", "--no-extras", "--steps", "2", "--warmup", "0",
                                      "--cases", "1", "--chunk", "64"])
    bench.main()
    rec = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline"):
        assert key in rec, key
    assert rec["n_gpus"] == 1 and rec["steps"] == 2 and rec["warmup"] == 0
    assert rec["value"] > 0 and rec["unit"] == "MLUPS" and rec["higher_is_better"] is True
    assert rec["dtype"] == "f32" and rec["vs_baseline"] is None
    assert "1024x1024" in rec["config"]["workload"]
    rf = rec["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == bench.PEAK_HBM_GBS
    assert rf["achieved"] > 0 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert rf["steps_per_launch"] >= 1 and rf["avg_launch_us"] > 0
    assert "traffic" in rf and "traffic_frac" in rf and "valu_frac" in rf
    # a fraction of a real ceiling: the launch's own minimum bytes over its duration
    assert rf["min_bytes_per_launch"] == 72 * 1024 * 1024 and 0 < rf["frac"] <= 1.0
    assert rf["effective_gbs"] == pytest.approx(rf["achieved"] * rf["steps_per_launch"], rel=1e-3)

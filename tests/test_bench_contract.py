"""bench.py's command-line contract on a machine without a GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_cpu_oracle_leg_reports_cores_and_sample():
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-oracle-only",
                        "--cpu-seconds", "0.5"], capture_output=True, text=True, timeout=300,
                       env=env)
    assert r.returncode == 0, r.stderr
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["kind"] == "oracle" and rec["cores"] == 1 and rec["unit"] == "MLUPS"
    assert rec["value"] > 0 and "1024x1024" in rec["sample"]


def test_roofline_arithmetic():
    """The roofline fields of a fused launch: minimum bytes = 72 B per FP32 site
    per launch (populations in and out, force in) whatever the steps per
    launch; frac against 8 TB/s; the one-step byte model as effective_gbs."""
    sys.path.insert(0, ROOT)
    import bench
    rf = bench.roofline("fp32", 1 << 20, 40.0, 8, "k_stepN<float, 16, 8, 512, 0> (tile)", None)
    want = 72 * (1 << 20) / 40e-6 / 1e9
    assert rf["min_bytes_per_launch"] == 72 * (1 << 20)
    assert abs(rf["achieved"] - want) < 0.1 and abs(rf["frac"] - want / 8000.0) < 1e-4
    assert abs(rf["effective_gbs"] - 8 * want) < 1.0
    assert rf["traffic"] is None and rf["valu_frac"] is None
    assert bench.PEAK_VALU_LANE_OPS == 256 * 4 * 16 * 2.4e9

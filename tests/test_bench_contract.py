"""The benchmark's output contract: one JSON line carrying the fields its readers expect,
a roofline object whose fraction is its own achieved/peak, and the CPU oracle baseline."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert not [l for l in r.stdout.splitlines() if l.startswith("{")]


@pytest.mark.gpu
def test_bench_line_fields():
    steps, warmup = 20, 2
    r = subprocess.run([sys.executable, "bench.py", "--steps", str(steps), "--warmup", str(warmup),
                        "--no-compare", "--no-extras", "--cpu-budget", "2"],
                       cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == steps and d["warmup"] == warmup
    assert d["higher_is_better"] is True and d["scaling"] == "weak" and d["data"] == "synthetic"
    assert d["unit"] == "gp-steps/s" and d["value"] > 0.0
    # value is grid-point-steps per second of the timed steps
    assert abs(d["value"] - d["config"]["points"] * 1e3 / d["ms_per_step"]) <= 1e-9 * d["value"]
    # the default workload: 256x128 per electron in complex64 storage
    assert "workload" in d["config"] and d["config"]["points"] == (256 * 128) ** 2
    assert d["config"]["precision"] == "mixed" and d["dtype"] == "f64"
    rl = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rl, k
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) <= 1e-12
    # achieved = algorithmic bytes of one launch over the average launch duration
    assert abs(rl["achieved"] - rl["algorithmic_bytes_per_launch"] / rl["avg_launch_s"] / 1e9) <= 1e-9 * rl["achieved"]
    # four passes per step; the x passes also take the opening half step
    assert d["config"]["passes_per_step"] == 4
    assert steps <= rl["launches_timed"] <= steps + 1
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0.0 and cpu["cores"] >= 1

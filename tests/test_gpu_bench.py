"""The benchmark's output contract on the GPU: one JSON line with the metric,
the whole-job value, the stage kernel's roofline (with HBM traffic from the
committed counter profile) and, unless disabled, the oracle's host
baseline."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    """The default workload (what the driver runs), shortened."""
    r = subprocess.run([sys.executable, "bench.py", "--steps", "6", "--warmup", "2",
                        "--profile-steps", "3", "--no-cpu-baseline", "--no-learned"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip().startswith("{")]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 6 and d["warmup"] == 2
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert d["dtype"] == "f64" and d["config"]["workload"].startswith("c5")
    rl = d["roofline"]
    assert rl["bound"] == "alu" and rl["peak"] == 78.6 and 0 < rl["frac"] < 1
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-12
    sys.path.insert(0, ROOT)
    import bench
    tile = d["config"]["tile"]["variant"]
    if bench.measured_traffic(tile, 1.0) is not None:
        # counters were taken on this kernel source and tile
        assert rl["traffic"] is not None and rl["traffic"] > 0
    else:
        assert rl["traffic"] is None

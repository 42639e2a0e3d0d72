"""Host-side contract of bench.py (CPU only): one GPU only, and the HBM
traffic it reports comes from a counter profile taken on the kernel source
that is committed."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_counter_profile_matches_the_committed_stage_kernel():
    b = _bench()
    with open(b.COUNTERS) as f:
        c = json.load(f)
    assert c["source_sha256"] == b.kernel_source_hash(), \
        "stage kernel sources changed since the counters in profiles/ were taken"
    for v, rec in c["variants"].items():
        assert rec["fetch_bytes_per_cell"] > 0 and rec["write_bytes_per_cell"] > 0, v


def test_traffic_only_for_profiled_variants():
    b = _bench()
    with open(b.COUNTERS) as f:
        c = json.load(f)
    v = next(iter(c["variants"]))
    rec = c["variants"][v]
    t = b.measured_traffic(int(v), 1000.0)
    assert t == (rec["fetch_bytes_per_cell"] + rec["write_bytes_per_cell"]) * 1000.0
    assert b.measured_traffic(10, 1000.0) is None      # a variant never profiled
    assert b.measured_traffic(None, 1000.0) is None


def test_algorithmic_bytes_per_cell_stage():
    b = _bench()
    # stage 1 reads U^n and writes the output; stages 2-3 also read the stage input
    assert b.bytes_per_cell_stage(2, 1) == 2 * 4 * 8
    assert b.bytes_per_cell_stage(2, 2) == 3 * 4 * 8
    assert b.bytes_per_cell_stage(3, 3) == 3 * 5 * 8

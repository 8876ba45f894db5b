"""Host-side checks of bench.py: the one-GPU refusal and the currency of the
committed HBM traffic counters (no GPU needed)."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    return bench


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_committed_traffic_counters_match_the_kernel_source():
    # The PMC summary records a hash of the GEMM source it was measured on;
    # bench.py reports its traffic only while that hash is current.
    bench = load_bench()
    t = bench.traffic_from_profiles(None, None)
    assert t is not None and 6 * 2 ** 30 < t < 1e12

"""Host-side behaviour of bench.py (no GPU): it refuses more than one GPU
before touching a device, and the HBM traffic it reports comes only from a
committed profile of the same kernel source."""
import importlib.util
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
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_from_a_matching_profile():
    b = _bench()
    # no profile for this kernel name: nothing reported
    assert b.measured_traffic("c2", "no_such_kernel") == (None, None)
    # a workload without a profile tag: nothing reported
    assert b.measured_traffic("no_such_config", "k_column") == (None, None)
    # the committed profile: a positive byte count when its source hash
    # matches the kernel file, None (with the file named) otherwise
    t, src = b.measured_traffic("c2", "k_column")
    assert src == os.path.join("profiles", "k_column_N200_beta7-4_K2048_secant.txt")
    assert t is None or t > 0

"""bench.py on the CPU: it parses, refuses more than one GPU with a message,
and its bookkeeping helpers are consistent."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_helpers():
    sys.path.insert(0, ROOT)
    import bench
    st = {"prop_linear2": 3, "prop_reified": 5, "prop_terms": 7}
    assert bench.algorithmic_bytes(st) == 3 * 16 + 5 * 24 + 7 * 8
    sha = bench.kernel_sha256()
    assert len(sha) == 64
    keys = {"kernel_sha256", "block", "desc_lds", "root_lds", "live", "occupancy", "dep",
            "fetch_bytes_per_node", "write_bytes_per_node", "profile"}
    for e in bench.PROFILED_TRAFFIC:
        assert set(e) == keys
        assert os.path.exists(os.path.join(ROOT, e["profile"]))
    # a shape that was never profiled reports no traffic
    st = {"block": 96, "desc_lds": 0, "root_lds": 0, "live": 0, "occupancy": 2, "dep": 0}
    assert bench.profiled_traffic(st, 1000) is None

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
    keys = {"workload", "kernel_sha256", "block", "desc_lds", "root_lds", "live", "occupancy",
            "dep", "fetch_bytes_per_node", "write_bytes_per_node", "profile"}
    for e in bench.PROFILED_TRAFFIC:
        assert set(e) == keys
        assert os.path.exists(os.path.join(ROOT, e["profile"]))
        st = {k: e[k] for k in ("block", "desc_lds", "root_lds", "live", "occupancy", "dep")}
        want = round((e["fetch_bytes_per_node"] + e["write_bytes_per_node"]) * 1000)
        if e["kernel_sha256"] == sha:
            assert bench.profiled_traffic(st, 1000, e["workload"]) == want
        # the same shape on another workload was not profiled
        assert bench.profiled_traffic(st, 1000, "another_workload") is None
    # a shape that was never profiled reports no traffic
    st = {"block": 96, "desc_lds": 0, "root_lds": 0, "live": 0, "occupancy": 2, "dep": 0}
    assert bench.profiled_traffic(st, 1000, "rcpsp_mixed_30_60_90tasks_4res_batch256") is None


def test_bench_roofline_and_cpu_baseline():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2207_12116_amd import instances as I
    peaks = {"read_GBs": 100.0, "atomic_Gops": 10.0}
    r = bench.roofline(50e9, 2e9, 1.0, peaks)
    assert r["achieved"] == 50.0 and r["frac"] == 0.5
    assert r["atomic_achieved"] == 2.0 and r["atomic_frac"] == 0.2
    # the CPU baseline builds a native copy of the oracle and times it in C
    cpu = bench.cpu_baseline({30: [I.rcpsp(30, s) for s in range(2)], 60: [I.rcpsp(60, 1)]}, 2,
                             "test sample", scale=0.1)
    assert cpu["cores"] == 2 and cpu["value"] > 0 and cpu["nproc"] >= 1
    assert cpu["single_core"]["value"] > 0

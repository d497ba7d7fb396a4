"""Host-side checks of bench.py (no GPU): it refuses more than one GPU with a
message, names the decode kernels as the profiler does, and takes HBM
traffic only from a counter summary of the current decode sources, the same
workload and the same kernel."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single" in r.stderr
    assert r.stdout == ""


def test_kernel_names():
    assert bench.kernel_name(1, 2048, 0) == "gc_wave_kernel<2048, 1, 2>"
    assert bench.kernel_name(4, 4096, 2) == "gc_wave_kernel<4096, 4, 0>"
    assert bench.kernel_name(0, 1024, 1) == "gc_wave_kernel<1024, 0, 2>"


def summary():
    kv = {}
    with open(bench.TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def test_traffic_only_for_the_profiled_sources_workload_and_kernel():
    kv = summary()
    units, kernel = int(kv["workload_units"]), kv["kernel"]
    got = bench.read_traffic(units, kernel)
    if kv["decode_sources_sha256"] == bench.decode_sources_sha256():
        assert got == float(kv["hbm_bytes_per_launch"])
    else:
        assert got is None          # stale summary: traffic is reported as null
    assert bench.read_traffic(units + 1, kernel) is None
    assert bench.read_traffic(units, "gc_wave_kernel<9999, 9, 9>") is None

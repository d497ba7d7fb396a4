"""Host-side checks of bench.py (no GPU): it refuses more than one GPU with a
message, names the decode kernels as the profiler does, and takes HBM
traffic only from a counter summary of the current decode sources, the same
workload, the same kernel and a plan that gives that kernel the same
algorithmic bytes."""
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


def summary(path):
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def test_traffic_only_for_the_profiled_sources_workload_and_kernel():
    found = 0
    for wl in bench.WORKLOADS:
        path = bench.traffic_file(wl)
        if not os.path.exists(path):
            assert bench.read_traffic(wl, 100000, "gc_wave_kernel<2048, 1, 2>", 1) is None
            continue
        found += 1
        kv = summary(path)
        units, kernel, alg = int(kv["workload_units"]), kv["kernel"], int(kv["algorithmic_bytes_per_launch"])
        got = bench.read_traffic(wl, units, kernel, alg)
        if kv["decode_sources_sha256"] == bench.decode_sources_sha256():
            assert got == float(kv["hbm_bytes_per_launch"])
        else:
            assert got is None          # stale summary: traffic is reported as null
        assert bench.read_traffic(wl, units + 1, kernel, alg) is None
        assert bench.read_traffic(wl, units, "gc_wave_kernel<9999, 9, 9>", alg) is None
        # another plan (a different packed-list threshold) gives the kernel other bytes
        assert bench.read_traffic(wl, units, kernel, alg + 4) is None
    assert found >= 1


def test_variant_table_covers_every_codec_variant():
    from paper_1502_01916_amd import gc
    names = [v[0] for v in bench.all_variants(gc)]
    assert len(names) == len(set(names)) == 15    # Simple, ten Group-Scheme, AFOR, PFD, BP128, VSE
    assert sum(1 for n in names if n.startswith("gsc-")) == 10

"""Builds libgc.so in-tree with hipcc for gfx950.

    python -m paper_1502_01916_amd.build

Every HIP source is compiled with packed-FP32 instruction selection turned
off; the host pass warns that it does not know that target feature, which is
harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libgc.so")

SOURCES = ["encode.cpp", "runtime.cpp", "decode.hip", "blocks.hip", "mlp.hip", "noalloc.hip", "encode_gpu.hip", "query.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-Wall"]


def _compile(src: str) -> subprocess.Popen:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True), obj


def build(verbose: bool = False) -> str:
    """Compiles every source and links libgc.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = [(s, *_compile(s)) for s in srcs]
    objs, errors = [], []
    for src, proc, obj in jobs:
        out, _ = proc.communicate()
        noise = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
        if proc.returncode != 0:
            errors.append("%s:\n%s" % (src, "\n".join(noise)))
        elif verbose and noise:
            print("\n".join(noise), file=sys.stderr)
        objs.append(obj)
    if errors:
        raise RuntimeError("libgc build failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp, "-lpthread"]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("libgc link failed:\n" + res.stdout)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

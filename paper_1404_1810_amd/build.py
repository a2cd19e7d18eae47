"""Build the gfx950 shared library ``libamqft.so`` in-tree with hipcc.

Usage: ``python -m paper_1404_1810_amd.build``.  Every HIP source is compiled
for gfx950 only, with packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libamqft.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["amqft_lds.hip", "amqft_fast.hip", "amqft_kA.hip", "amqft_kB.hip", "amqft_kLT.hip", "amqft_multipass.hip", "amqft_static.hip", "amqft_api.cpp"]
HEADERS = ["amqft_device.h", "amqft_internal.h", "amqft_levels.h", "amqft_leaf.h", "amqft_kA_passes.h", "amqft_kB_passes.h",
           "amqft_iplayout.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    "-std=c++17", "-O3", "-fPIC", "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _compile_one(src: str, obj: str) -> None:
    cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.check_call(cmd)


def build(verbose: bool = True, jobs: int | None = None) -> str:
    """Compile all sources (always) and link libamqft.so; returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    t0 = time.time()
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd)))
    for src, p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed on " + src)
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0), file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()

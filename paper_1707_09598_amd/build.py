"""Build libigasg.so (host plan + gfx950 kernels) in-tree with hipcc.

All HIP code is compiled for gfx950 only, with packed FP32 instructions
disabled (-target-feature -packed-fp32-ops).  Host-only C++ (plan, eigen
solver) is compiled with g++.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libigasg.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-march=x86-64-v2", "-Wall", "-pthread", f"-I{INCLUDE}"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    if not force and os.path.exists(OUT):
        return OUT
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in sorted(os.listdir(CSRC)):
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        if src.endswith(".cpp"):
            jobs.append((["g++", *CXX_FLAGS, "-c", path, "-o", obj], obj))
        elif src.endswith(".hip"):
            jobs.append(([HIPCC, *HIP_FLAGS, "-c", path, "-o", obj], obj))
    # translation units are independent: compile them concurrently
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "8")), os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda j: _run(j[0]), jobs))
    objs = [obj for _, obj in jobs]
    tmp = OUT + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(force=True)
    sys.exit(0)

"""Build libcpra.so in-tree for gfx950 (hipcc cross-compiles without a GPU).

Usage: python -m paper_2402_05283_amd.build  (or build() from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcpra.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-variable",
    "-Wno-unused-but-set-variable",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    r = subprocess.run(cmd, cwd=HERE, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


SOURCES = ["cpra.hip", "inst_64.hip", "inst_128.hip", "inst_192.hip", "inst_256.hip", "inst_384.hip", "inst_512.hip",
           "inst_1024.hip"]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every translation unit for gfx950 (in parallel) and link libcpra.so."""
    from concurrent.futures import ThreadPoolExecutor

    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    os.makedirs(BUILD_DIR, exist_ok=True)
    host_o = os.path.join(BUILD_DIR, "host_geom.o")
    cmds = [["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-c",
             os.path.join(CSRC, "host_geom.cpp"), "-o", host_o]]
    objs = [host_o]
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

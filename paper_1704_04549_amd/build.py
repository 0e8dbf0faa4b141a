"""Build the HIP library libkp.so for gfx950 (and the host build used by CPU tests).

Usage: python -m paper_1704_04549_amd.build   (or build() from __graft_entry__)

Every call recompiles.  Objects go to paper_1704_04549_amd/_build/, the
library to paper_1704_04549_amd/libkp.so.  The host-check library (the
per-element routines of elem_ops.h built for the CPU with a one-thread team,
loaded only by the CPU tests) goes to tests/_native/libkp_hostcheck.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libkp.so")
HOSTCHECK = os.path.join(ROOT, "tests", "_native", "libkp_hostcheck.so")

HIP_SOURCES = ["kernels.hip", "apply_mfma.hip", "rank3.hip", "learned.hip", "mixed.hip", "krylov.hip", "bj.hip", "mlp.hip",
               "quad.hip", "sys.hip", "apply_small.hip"]
CPP_SOURCES = ["kp_api.cpp", "mlp_api.cpp", "mixed_api.cpp", "tables.cpp", "quad_tables.cpp", "sys_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
# packed FP32 instructions are kept out of every kernel
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in HIP_SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([HIPCC, *COMMON, *DEVICE, "-x", "hip", "-c", path, "-o", obj])
    for src in CPP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        # host code (the C ABI); hipcc compiles it as HIP, so it targets gfx950 too
        jobs.append([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        list(ex.map(_run, jobs))
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    # host build of the per-element routines for the CPU tests
    os.makedirs(os.path.dirname(HOSTCHECK), exist_ok=True)
    cxx = shutil.which("g++") or "g++"
    _run([cxx, "-O2", "-std=c++17", "-shared", "-fPIC", f"-I{CSRC}", "-o", HOSTCHECK + ".tmp",
          os.path.join(CSRC, "hostcheck.cpp"), os.path.join(CSRC, "tables.cpp"),
          os.path.join(CSRC, "quad_tables.cpp")])
    os.replace(HOSTCHECK + ".tmp", HOSTCHECK)
    if verbose:
        print("built", LIB, "and", HOSTCHECK)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

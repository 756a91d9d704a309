"""Build libqs.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2609_19147_amd.build  (or build() from Python).
Every source is compiled on each call; objects go to ``_build/``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libqs.so")
# standalone streaming-ceiling probe (bench.py runs it beside the benchmark)
PROBE_SRC = os.path.join(CSRC, "ceiling_probe.hip")
PROBE = os.path.join(PKG, "ceiling_probe")

SOURCES = ["planner.cpp", "api.cpp", "runtime.cpp", "adjoint.cpp", "batch.cpp",
           "k_tile.hip", "k_dense.hip", "k_sample.hip", "k_stream.hip", "k_plain.hip", "k_reduce.hip"]

ARCH = os.environ.get("QS_OFFLOAD_ARCH", "gfx950")
# Packed FP32 instructions are kept out of every kernel.
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
           "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *DEVICE_FLAGS, *extra,
           "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build_probe() -> str:
    tmp = PROBE + ".tmp"
    cmd = [hipcc(), "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", *DEVICE_FLAGS, PROBE_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for ceiling_probe.hip:\n{r.stderr[-6000:]}")
    os.replace(tmp, PROBE)
    return PROBE


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES) + 1)) as ex:
        probe = ex.submit(build_probe)
        objs = list(ex.map(lambda s: _compile(s, list(extra)), SOURCES))
        probe.result()
    tmp = LIB + ".tmp"
    # rocTX for the profiler ranges (rocprofiler-sdk's marker library)
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           f"-L{ROCM}/lib", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

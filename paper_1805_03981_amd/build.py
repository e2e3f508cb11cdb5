"""Builds libdgw.so (the solver) and libdgw_ceilings.so (device ceiling
microbenchmarks) for gfx950 in-tree with hipcc.

Run as `python -m paper_1805_03981_amd.build` or call build().  Objects go
to _build/ at the repository root; the shared libraries are written next to
this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libdgw.so")
OUT_CEIL = os.path.join(HERE, "libdgw_ceilings.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["abi.hip", "serve.hip", "setup.cpp", "exterior.hip", "inst_d2_f64.hip", "inst_d2_f32.hip",
           "inst_d3_f64.hip", "inst_d3_f32.hip"]
CEIL_SOURCES = ["ceilings.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall", "-Wno-unused-function"]
# hipcc: no packed FP32 instructions anywhere (they are unreliable on this part)
DEVICE_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-ffp-contract=fast"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD_DIR, src + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip", *DEVICE_FLAGS, *COMMON, "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, out):
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    shutil.move(tmp, out)


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every source and link libdgw.so and libdgw_ceilings.so;
    returns the path of libdgw.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES + CEIL_SOURCES))
    _link(objs[:len(SOURCES)], OUT)
    _link(objs[len(SOURCES):], OUT_CEIL)
    if verbose:
        print(f"built {OUT} and {OUT_CEIL}", file=sys.stderr)
    return OUT


if __name__ == "__main__":
    build(verbose=True)

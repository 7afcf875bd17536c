"""Build the HIP shared library libhpdg.so for gfx950, in-tree.

Usage: python -m paper_2009_01287_amd.build   (or build() from Python)
Host setup sources are compiled as C++, the kernels and the C ABI as HIP.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhpdg.so")
OBJ = os.path.join(HERE, "_build")
HOST_SRC = ["basis.cpp", "mesh.cpp", "setup_ops.cpp", "amg.cpp"]
HIP_SRC = ["capi.hip"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compile failed: " + " ".join(cmd))
    return r


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = []
    for s in HOST_SRC:
        jobs.append([hipcc, *COMMON, "-c", os.path.join(CSRC, s), "-o", os.path.join(OBJ, s + ".o")])
    for s in HIP_SRC:
        jobs.append([hipcc, *COMMON, *HIP_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, s),
                     "-o", os.path.join(OBJ, s + ".o")])
    with ThreadPoolExecutor(max_workers=4) as ex:
        for r in ex.map(_run, jobs):
            if verbose and r.stderr:
                sys.stderr.write(r.stderr)
    objs = [os.path.join(OBJ, s + ".o") for s in HOST_SRC + HIP_SRC]
    tmp = OUT + ".tmp"
    _run([hipcc, "-shared", "--offload-arch=gfx950", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))

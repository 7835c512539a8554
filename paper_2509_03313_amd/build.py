"""Build libgsbs.so (HIP kernels for gfx950 + host scheduler + C ABI) in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libgsbs.so")

ARCH = "gfx950"
# FP32 results must not depend on contraction; packed FP32 ops are kept off.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-I", INCLUDE, "-I", CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


SOURCES = (("kernels.hip", True), ("mlp.hip", True), ("surrogate.hip", True), ("numodes.hip", True), ("ssa.hip", True), ("spurs.hip", True), ("api.cpp", False),
           ("mlp_api.cpp", False))


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    objs, procs = [], []
    for src, dev in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [hipcc, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON
        if dev:
            cmd += DEVICE
        else:
            cmd += ["-D__HIP_PLATFORM_AMD__"]
        if verbose:
            print(" ".join(cmd))
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

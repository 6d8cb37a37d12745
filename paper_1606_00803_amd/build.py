"""Build ``liblms.so`` (host C++ + HIP kernels for gfx950) in-tree.

    python -m paper_1606_00803_amd.build

Host sources are compiled with g++, the HIP source with hipcc for gfx950;
all with -ffp-contract=off (no fused multiply-add: the arithmetic is exactly
the IEEE operations in the source).  Packed-FP32 instructions are disabled in
device code.  Objects go to ``_build/`` at the repository root.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "liblms.so")
ARCH = os.environ.get("LMS_OFFLOAD_ARCH", "gfx950")

HOST_SRC = ["lms_host.cpp", "lms_api.cpp"]
HIP_SRC = ["lms_device.hip", "lms_reorder.hip"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wextra", f"-I{INC}", f"-I{CSRC}"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    """Compile every source and link ``liblms.so``; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for s in HOST_SRC:
        o = os.path.join(BUILD, s + ".o")
        _run(["g++", *COMMON, "-pthread", "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    hipcc = _hipcc()
    for s in HIP_SRC:
        o = os.path.join(BUILD, s + ".o")
        _run([hipcc, *COMMON, f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wno-unused-command-line-argument",
              "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-pthread", "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)

"""Compile the oracle's C sweeps (``sweep.c``) into ``_sweep.so`` with gcc.

Test infrastructure: part of the oracle, never of the library.  Flags:
-O2 and -ffp-contract=off (no fused multiply-add: every operation in the C
source is the IEEE operation written), -fopenmp for the optional static
schedule of the Jacobi sweep.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sweep.c")
LIB = os.path.join(HERE, "_sweep.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-std=c99", "-fopenmp", "-Wall", "-Wextra"]


def build(force: bool = False) -> str:
    """Build ``_sweep.so`` (always when ``force``, else only when stale)."""
    if (not force and os.path.exists(LIB)
            and os.path.getmtime(LIB) >= os.path.getmtime(SRC)):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))

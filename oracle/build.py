"""Compile the CPU oracle into oracle/liboracle.so (plain C, gcc).

The library the tests load is built for the generic x86-64 target, so the
copy that travels with the repository runs on any host.  The CPU baseline of
the benchmark times a second copy built with -march=native on the host that
runs it (build(native=True, out=...)); the sources are the same.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["propagate.c", "search.c", "brute.c", "learn.c", "timing.c", "fprop.c"]


def build(verbose: bool = False, native: bool = False, out: str | None = None) -> str:
    out = out or os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3"] + (["-march=native"] if native else []) + [
        "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
        # fprop.c changes the rounding mode between operations
        "-frounding-math", "-ffp-contract=off",
        "-o", tmp] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

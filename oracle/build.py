"""Compile the CPU oracle (plain C) into oracle/liboracle.so with gcc.

Test infrastructure: the library built here is loaded only by the tests, the package's smoke
check and the benchmark's CPU-baseline leg.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gom_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, out: str = LIB, native: bool = False) -> str:
    """Always recompiles.  The in-tree library is portable -O2 (it travels to other hosts);
    native=True adds -march=native for a copy built on the host that times it.  OpenMP spreads
    a colour class's solutions over threads when a run asks for more than one worker."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", *(["-march=native"] if native else []), SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

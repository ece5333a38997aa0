"""Compile the C oracle (test infrastructure) into oracle/liboracle.so with gcc.

Flags: -O2 -ffp-contract=off so that every floating-point operation rounds once,
in source order, and -fopenmp for the pencil-parallel loop of the sweeps and the
paper's other OpenMP schemes (their results do not depend on the thread count).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["hydro_oracle.c", "mlp_oracle.c", "openmp_schemes.c"]
OUT = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared",
          "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = OUT + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

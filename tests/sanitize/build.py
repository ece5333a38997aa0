"""Build the oracle driver (oracle_driver.c + the oracle's C sources) with the
compiler sanitizers, for the CPU test suite.  Test infrastructure.

  asan   gcc: AddressSanitizer + UndefinedBehaviorSanitizer, abort on the first
         report (-fno-sanitize-recover=all), libgomp.
  tsan   clang from the ROCm LLVM with its OpenMP runtime (libomp):
         ThreadSanitizer.  Run it with OMP_TOOL_LIBRARIES pointing at the
         runtime's Archer tool (ARCHER_LIB), which tells ThreadSanitizer about
         OpenMP's own barriers and task dependencies; without it every
         implicit barrier of the runtime reads as a race.

Both keep the oracle's floating-point flags (-ffp-contract=off) so the
schemes' bitwise checks mean the same as in the regular build.
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ORACLE = os.path.join(ROOT, "oracle")
SOURCES = [os.path.join(HERE, "oracle_driver.c")] + [
    os.path.join(ORACLE, s) for s in ("hydro_oracle.c", "mlp_oracle.c", "openmp_schemes.c")]
LLVM = "/opt/rocm/llvm"
CLANG = os.path.join(LLVM, "bin", "clang")
ARCHER_LIB = os.path.join(LLVM, "lib", "libarcher.so")

COMMON = ["-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fno-omit-frame-pointer", f"-I{ORACLE}"]


def tsan_available() -> bool:
    return os.path.exists(CLANG) and os.path.exists(ARCHER_LIB)


def build(kind: str, outdir: str, verbose: bool = False) -> str:
    out = os.path.join(outdir, f"oracle_driver_{kind}")
    if kind == "asan":
        cmd = [shutil.which("gcc") or "gcc", *COMMON, "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", *SOURCES, "-lm", "-o", out]
    elif kind == "tsan":
        cmd = [CLANG, *COMMON, "-fsanitize=thread", *SOURCES, "-lm", "-o", out,
               f"-Wl,-rpath,{os.path.join(LLVM, 'lib')}"]
    else:
        raise ValueError(kind)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    return out

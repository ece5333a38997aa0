"""Compile the plain-C example of the C ABI (tests/c_abi/step_blast.c) against
the in-tree libhydro.so and the HIP runtime; the binary finds the library
through a relative run path."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
BIN = os.path.join(HERE, "step_blast")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{os.path.join(ROCM, 'include')}",
           os.path.join(HERE, "step_blast.c"), "-o", BIN + ".tmp",
           f"-L{os.path.join(ROOT, 'paper_2106_13465_amd')}", "-lhydro",
           f"-L{os.path.join(ROCM, 'lib')}", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2106_13465_amd", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    print(build(verbose=True))

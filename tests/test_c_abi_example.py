"""The C ABI from plain C (tests/c_abi/step_blast.c): built against the
in-tree library without Python in the loop; on the GPU its result equals the
FP64 oracle's."""
import importlib.util
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
BIN = os.path.join(HERE, "c_abi", "step_blast")
LIB = os.path.join(os.path.dirname(HERE), "paper_2106_13465_amd", "libhydro.so")


def _ensure_built():
    if not os.path.exists(BIN):
        if not os.path.exists(LIB):
            pytest.skip("libhydro.so not built")
        spec = importlib.util.spec_from_file_location(
            "c_abi_example_build", os.path.join(HERE, "c_abi", "build.py"))
        c_build = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(c_build)
        c_build.build()
    return BIN


def test_c_example_links_against_the_library():
    b = _ensure_built()
    out = subprocess.run(["ldd", b], capture_output=True, text=True, check=True).stdout
    assert "libhydro.so" in out and "not found" not in out


@pytest.mark.gpu
def test_c_example_matches_oracle(orc, tmp_path):
    from paper_2106_13465_amd import inputs

    b = _ensure_built()
    out = tmp_path / "state.bin"
    res = subprocess.run([b, str(out)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    got = np.fromfile(out, dtype=np.float64).reshape(4, 64, 64)
    ref = inputs.blast_corner(64)
    c = orc.cfg(bc=orc.BC_REFLECT)
    for _ in range(3):
        orc.step(ref, c)
    err = max(np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max() for k in range(4))
    assert err <= 1e-12, err
    tot = [float(v) for v in res.stdout.split()[1:5]]
    np.testing.assert_allclose(tot[0], orc.totals(ref)[0], rtol=1e-13)

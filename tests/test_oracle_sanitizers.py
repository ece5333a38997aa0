"""The CPU oracle under the compiler sanitizers (CPU only): every solver path,
the network oracle and the paper's three OpenMP schemes with AddressSanitizer
and UndefinedBehaviorSanitizer; the fine- and coarse-grain schemes with
ThreadSanitizer, which checks that the coarse-grain barrier (a thread writes a
pencil segment only after both neighbours have read that pencil, paper
Section 3) orders every neighbour's READ before the WRITE."""
import importlib.util
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "sanitize", "build.py")

pytestmark = pytest.mark.skipif(not os.path.exists(BUILD), reason="sanitizer driver not present")


def _builder():
    spec = importlib.util.spec_from_file_location("sanitize_build", BUILD)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _run(exe, mode, env):
    res = subprocess.run([exe, mode], capture_output=True, text=True, timeout=600, env=env)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert f"{mode}: ok" in res.stdout, out[-4000:]
    assert "Sanitizer" not in res.stderr, out[-4000:]
    assert "runtime error" not in res.stderr, out[-4000:]


def test_oracle_asan_ubsan(tmp_path):
    b = _builder()
    exe = b.build("asan", str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    _run(exe, "all", env)


def test_oracle_tsan_schemes(tmp_path):
    b = _builder()
    if not b.tsan_available():
        pytest.skip("clang with ThreadSanitizer and the OpenMP Archer tool not found")
    exe = b.build("tsan", str(tmp_path))
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:ignore_noninstrumented_modules=1",
               OMP_TOOL_LIBRARIES=b.ARCHER_LIB)
    _run(exe, "threads", env)

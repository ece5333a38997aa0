"""The C-ABI library loads and exports every function include/*.h declares
(no device calls: runs without a GPU)."""
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for path in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^[\w \*]+?\b(hydro_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("hydro_create", "hydro_compute_dt", "hydro_sweep", "hydro_step",
                 "hydro_conserved_totals"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2106_13465_amd import _lib

    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\b(hydro_\w+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_binding_signatures_cover_the_header():
    from paper_2106_13465_amd import _lib

    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_no_cpu_fallback(monkeypatch, tmp_path):
    """Without the built library the binding fails loudly."""
    from paper_2106_13465_amd import _lib

    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asking for more exits with status 2 and a
    message, before touching any device."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

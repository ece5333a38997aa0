"""Host logic of bench.py: the kernel-code hash that ties the committed counter
summaries to the kernels they measured."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_of_strips_comments_and_layout_only():
    src = ('int a = 1;  // trailing "comment"\n/* block\n   comment */ const char* s = "a // b";\n'
           "char c = '/'; x = y / z; /* \"*/ w;\n")
    assert bench.code_of(src) == ('int a = 1; const char* s = "a // b"; char c = \'/\'; '
                                  "x = y / z; w;")
    # a changed token changes the code, a changed comment does not
    assert bench.code_of("x = y + 1; // one") == bench.code_of("x = y + 1;   // two\n")
    assert bench.code_of("x = y + 1;") != bench.code_of("x = y + 2;")


def test_committed_counter_summaries_match_the_kernel_code():
    h = bench.kernel_source_hash()
    names = list(bench.PMC_SUMMARY.values()) + ["sweep_fourier_blasts_8192_valu.json"]
    for name in names:
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        assert rec["kernel_source_hash"] == h, name

"""Host-side helpers of bench.py: the code hash that decides whether the
committed HBM-traffic counters still describe the pair kernels, and the
refusal of more than one GPU."""
import os
import subprocess
import sys

import bench


def test_code_only_strips_comments_and_layout():
    src = ('int a = 1;  // trailing comment\n'
           '/* block\n   comment */ const char* s = "x // not a comment /* nor this */";\n'
           "char q = '\\''; char r = '/';   int b = a / 2;\n")
    assert bench.code_only(src) == (
        'int a = 1; const char* s = "x // not a comment /* nor this */"; '
        "char q = '\\''; char r = '/'; int b = a / 2;")


def test_code_only_sees_code_edits_only():
    base = "double f(double x) {\n    // scale\n    return 2.0 * x;   /* doubled */\n}\n"
    recommented = "double f(double x)\n{\n    /* twice x */ return 2.0 * x;  // same code\n}\n"
    edited = "double f(double x) {\n    // scale\n    return 3.0 * x;\n}\n"
    assert bench.code_only(base) == bench.code_only(recommented)
    assert bench.code_only(base) != bench.code_only(edited)


def test_library_source_hash_is_stable():
    h = bench.library_source_hash()
    assert len(h) == 64 and h == bench.library_source_hash()


def test_more_than_one_gpu_is_refused():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""

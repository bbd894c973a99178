"""Host-side helpers of bench.py: the code hash that decides whether the
committed HBM-traffic counters still describe the pair kernels, the clock
sampler of the timed region, and the refusal of more than one GPU."""
import os
import subprocess
import sys
import time
import types

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


def _fake_torch(rates):
    """A stand-in whose cuda.clock_rate returns the given values in turn
    (then the last one), or raises when rates is None."""
    it = iter(rates or [])
    last = [None]

    def clock_rate(dev=None):
        if rates is None:
            raise RuntimeError("no amd-smi")
        last[0] = next(it, last[0])
        return last[0]
    return types.SimpleNamespace(cuda=types.SimpleNamespace(clock_rate=clock_rate))


def test_clock_sampler_averages_the_region():
    s = bench.ClockSampler(_fake_torch([2000, 2100, 2300]), period=0.01)
    with s:
        time.sleep(0.1)
    # the first query (before the region) is not a sample
    assert s.ok and len(s.samples) >= 2
    assert set(s.samples) <= {2100.0, 2300.0}
    assert s.mean() == round(sum(s.samples) / len(s.samples))


def test_clock_sampler_without_the_query_reports_none():
    s = bench.ClockSampler(_fake_torch(None), period=0.01)
    with s:
        time.sleep(0.02)
    assert s.mean() is None

"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

1. The oracle, built by gcc with -fsanitize=address,undefined (every
   undefined-behaviour report fatal), runs its pin suites.
2. The library's host runtime -- argument validation, workspace layouts,
   launch-shape choice, tuning table, batch and pool planning, the
   allocation-free call's refusals -- built by hipcc with the sanitizers on
   the host side only (device code is built as usual), runs the host-side
   ABI tests, which make no GPU call.

Each runs in a subprocess with the matching sanitizer runtime preloaded (the
Python interpreter itself is not instrumented); leak checking is off
because the interpreter keeps its allocations until exit.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_pytest(env, files, timeout):
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow", *files],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-fPIC", "-shared", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "oracle", "zm_oracle.c"), "-o", str(lib), "-lm"], check=True)
    runtime = subprocess.run(["gcc", "-print-file-name=libasan.so"], check=True,
                             capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", ZMO_ORACLE_LIB=str(lib),
               OMP_NUM_THREADS="4")
    files = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_pins.py", "test_oracle_vterms.py", "test_oracle_cutoff.py",
              "test_oracle_free.py", "test_oracle_loworder.py", "test_oracle_medium.py",
              "test_oracle_bruteforce.py")]
    _run_pytest(env, files, timeout=900)


def _clang_asan_runtime():
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.slow
def test_host_runtime_under_asan_and_ubsan(tmp_path):
    runtime = _clang_asan_runtime()
    if runtime is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "zm_lib_build_san", os.path.join(ROOT, "paper_2406_05490_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    lib = str(tmp_path / "libzm_san.so")
    # sanitizers on the host side only: device code is unaffected
    flags = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
             "-fno-omit-frame-pointer"]
    mod.build(out=lib, extra_flags=flags, obj_dir=str(tmp_path))
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", ZM_LIBRARY=lib)
    _run_pytest(env, [os.path.join(ROOT, "tests", "test_abi_cpu.py")], timeout=900)

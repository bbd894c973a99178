"""Build libzm.so (HIP kernels + host runtime) in-tree for gfx950.

    python paper_2406_05490_amd/build.py [-v] [--asm DIR]

Run it as a script (or load it by file path): importing the package itself
loads libzm.so, which is what this builds.

Packed-FP32 instruction selection is disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libzm.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("zm_kernels.hip", "zm_batch.hip", "zm_api.hip", "zm_batch_api.hip", "zm_tune.hip",
            "zm_pool_api.hip", "zm_cutoff.hip", "zm_lowfft.hip", "zm_noalloc.hip")]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", INCLUDE, "-I", CSRC,
]


def build(verbose: bool = False, asm_dir: str | None = None, defines=(), out: str = LIB,
          extra_flags=(), obj_dir: str | None = None) -> str:
    """Compile and link; `defines` are extra -D macros (tuning builds), `out`
    the library path, `extra_flags` more compile and link flags (e.g. host-only
    sanitizers), `obj_dir` where the objects go (default: next to the
    sources)."""
    objs = []
    extra = [f"-D{d}" for d in defines] + list(extra_flags)
    tag = "_".join(d.replace("=", "") for d in defines)
    for src in SOURCES:
        obj = os.path.join(obj_dir or CSRC,
                           os.path.basename(src) + (f".{tag}" if tag else "") + ".o")
        cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
        if asm_dir:
            os.makedirs(asm_dir, exist_ok=True)
            acmd = [HIPCC, *FLAGS, *extra, "--cuda-device-only", "-S", src, "-o",
                    os.path.join(asm_dir, os.path.basename(src) + ".s")]
            subprocess.run(acmd, check=True)
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra_flags, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    asm = None
    if "--asm" in sys.argv:
        asm = sys.argv[sys.argv.index("--asm") + 1]
    build(verbose="-v" in sys.argv, asm_dir=asm)

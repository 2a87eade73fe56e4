"""Build ``libpspfft.so`` (HIP, gfx950) in-tree.

Usage: ``python -m paper_1106_0557_amd.build`` or ``build()`` from Python.
Every call recompiles (the build check compiles each time it is asked to).
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpspfft.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are disabled for every HIP compile.  The sign of a
# zero plays no part in the results, so x + 0 folds to x (the known-zero halves
# of padded lines cost no additions).
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-parameter", "-fno-signed-zeros",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

DEVICE_SOURCES = (["green.hip", "line_generic.hip", "noalloc.hip", "pass_f32_e32.hip"]
                  + [f"pass_{p}_e{e}.hip" for p in ("f32", "f64") for e in (16, 20, 24, 36)])
HOST_SOURCES = ["pspfft_runtime.cpp"]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True, jobs: int = 8) -> str:
    out_dir = tempfile.mkdtemp(prefix="pspfft_build_")
    objs = []
    procs = []
    for src in DEVICE_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        cmd = [HIPCC, f"--offload-arch={ARCH}", *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        cmd = [HIPCC, f"--offload-arch={ARCH}", *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, p in procs:
        if verbose:
            print("+", " ".join(cmd), flush=True)
        if p.wait() != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd))
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    for o in objs:
        os.unlink(o)
    os.rmdir(out_dir)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)

"""Build libadiwave.so (gfx950) in-tree with hipcc.

    python -m paper_2006_10142_amd.build          # compile
    python -m paper_2006_10142_amd.build --check  # print the command only
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libadiwave.so")
ARCH = os.environ.get("ADIWAVE_ARCH", "gfx950")

SOURCES = [os.path.join(CSRC, "adiwave.hip")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libadiwave.so)")


def command(out: str) -> list:
    return [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
            # keep packed-FP32 instructions out of the device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", INCLUDE, "-I", CSRC, "-o", out] + SOURCES


def build(verbose: bool = False) -> str:
    """Compile every source into libadiwave.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libadiwave.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    if "--check" in sys.argv:
        print(" ".join(command(LIB)))
    else:
        print(build(verbose=True))

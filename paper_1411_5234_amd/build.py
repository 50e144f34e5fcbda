"""Build libnbody.so (the HIP/gfx950 hot path) in-tree with hipcc.

    python -m paper_1411_5234_amd.build

Packed FP32 instructions are switched off (-packed-fp32-ops): the kernels are
written in scalar FP32/FP64 and the compiler must not pair them.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnbody.so")
SOURCES = ["api.hip", "force.hip", "force6.hip", "step.hip", "step6.hip", "groups.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags() -> list[str]:
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result", "-fopenmp"]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    """Compile every HIP source and link libnbody.so; returns the library path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + compile_flags() + (extra or []) + ["-shared", "-o", tmp] + \
        [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libnbody.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

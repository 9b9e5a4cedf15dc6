"""Builds librsos.so (the gfx950 HIP kernels and the C ABI of include/rsos.h)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "rsos.hip")
HDRS = [os.path.join(PKG, "csrc", f) for f in ("rsos_kernels.hpp", "rsos_host.hpp", "rsos_moments.hpp", "rsos_ms.hpp", "rsos_engine.inc", "rsos_ms.inc", "rsos_tune.inc")] + [
    os.path.join(ROOT, "include", "rsos.h")]
OUT = os.path.join(PKG, "librsos.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(OUT):
        newest = max(os.path.getmtime(p) for p in [SRC] + HDRS)
        if os.path.getmtime(OUT) >= newest:
            return OUT
    tmp = OUT + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(OUT)
    sys.exit(0)

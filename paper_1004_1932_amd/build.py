"""Build the HIP library libad.so in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
LIB = PKG / "libad.so"
SOURCES = [CSRC / "ad_kernels.hip", CSRC / "ad_dense.hip", CSRC / "ad_runtime.hip", CSRC / "ad_sa.hip",
           CSRC / "ad_noalloc.hip", CSRC / "ad_calib.hip"]
HEADERS = [CSRC / "ad_internal.h", CSRC / "ad_order.h", PKG.parent / "include" / "ad.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every FP64 expression is evaluated as written; FP32 FMAs are explicit
    "-ffp-contract=off", "-fno-fast-math",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # roctx ranges over the stepping and mobility calls
    "-lrocprofiler-sdk-roctx",
]


def build(verbose: bool = False) -> Path:
    """Compile every HIP source into libad.so (always recompiles)."""
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, *FLAGS, *map(str, SOURCES), "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

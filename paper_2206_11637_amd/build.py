"""Build the HIP libraries for gfx950 (in-tree): libpflbm.so (D3Q15 phase
field) and libpflbm_d3q27.so (the same sources with the D3Q27 phase lattice)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "pflbm.hip")
OUT = os.path.join(PKG, "libpflbm.so")
# build variants: output file and extra flags (the D3Q27 phase lattice holds
# 27 h per cell, so its FP32-arithmetic step and reverse step run 2 waves per
# SIMD instead of 3)
VARIANTS = {
    "d3q15": (OUT, []),
    "d3q27": (os.path.join(PKG, "libpflbm_d3q27.so"), ["-DPFLBM_PHASE_D3Q27", "-DPFLBM_F32_WAVES=2",
                                                           "-DPFLBM_ADJ_WAVES=2"]),
}

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # a * b + c is fused only where it is written as one expression: with the
    # default (fuse across statements) the compiler's choice of which product
    # to fuse followed the placement of code in branches, and the two
    # streaming schemes, or one scheme with and without its fast-wave branch,
    # stopped giving the same bits
    "-ffp-contract=on",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libpflbm.so)")


def build(verbose: bool = False, variants=("d3q15", "d3q27")) -> list:
    """Compile csrc/pflbm.hip into each variant's library next to this file
    (in parallel); returns their paths."""
    jobs = []
    for v in variants:
        out, extra = VARIANTS[v]
        cmd = [hipcc()] + HIPCC_FLAGS + extra + ["-o", out + ".tmp", SRC]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((out, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                           text=True)))
    errors = []
    for out, p in jobs:
        _, err = p.communicate()
        if p.returncode != 0:
            errors.append(f"hipcc failed for {os.path.basename(out)} ({p.returncode}):\n{err[-8000:]}")
        else:
            os.replace(out + ".tmp", out)
    if errors:
        raise RuntimeError("\n".join(errors))
    return [out for out, _ in jobs]


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

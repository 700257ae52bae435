"""Builds libgaps.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["capi.hip", "kernels.hip", "shower.hip", "shower_wave.hip", "obs.hip", "mlp.hip"]
LIB = os.path.join(HERE, "libgaps.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the parity contract: no floating-point contraction, IEEE FP64 throughout
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no machine-level loop-invariant code motion: hoisting constants and
    # kernel arguments out of the persistent shower loop holds them in
    # registers for its whole length (243 instead of 173 VGPRs)
    "-mllvm", "-disable-machine-licm",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    cmd = ["hipcc", *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp"]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)

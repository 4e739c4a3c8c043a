"""Builds libchess.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(_HERE, "csrc")
SOURCES = ["kernels.hip", "kernels_listed.hip", "learned.hip", "chess.cpp", "hostmath.cpp", "ssf.cpp"]
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def library_path() -> str:
    return os.path.join(_HERE, "libchess.so")


def build_library(verbose: bool = False) -> str:
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *[os.path.join(_CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))

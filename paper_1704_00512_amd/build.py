"""Builds libchess.so in-tree with hipcc for gfx950.

Each source is compiled to an object file in its own hipcc process (in
parallel), then the objects are linked into the shared library."""
from __future__ import annotations

import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(_HERE, "csrc")
SOURCES = ["kernels.hip", "kernels_listed.hip", "kernels_stat.hip", "learned.hip", "chess.cpp",
           "hostmath.cpp", "ssf.cpp"]
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def library_path() -> str:
    return os.path.join(_HERE, "libchess.so")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build_library(verbose: bool = False) -> str:
    out = library_path()
    tmp = out + ".tmp"
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(_CSRC, s))]
    with tempfile.TemporaryDirectory() as d:
        objs = [os.path.join(d, s + ".o") for s in srcs]
        cmds = [["hipcc", *HIPCC_FLAGS, "-c", os.path.join(_CSRC, s), "-o", o]
                for s, o in zip(srcs, objs)]
        with ThreadPoolExecutor(max_workers=min(8, len(cmds))) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))

"""Builds the HIP library libwrs.so (gfx950) in the package directory, and
libwrs_roofs.so, the benchmark's ceiling kernels (random gathers, Philox)."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libwrs.so")
ROOFS_LIB = os.path.join(HERE, "libwrs_roofs.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _hipcc(srcs, out, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    _hipcc(sources(), LIB, verbose)
    _hipcc([os.path.join(HERE, "roofs", "wrs_roofs.hip")], ROOFS_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the package's native libraries in-tree.

libcsbfs.so  -- HIP kernels + C ABI (hipcc, gfx950 only)
librmat.so   -- seeded input generator (gcc, OpenMP)
"""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(REPO, "include"),
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_rmat(verbose: bool = False) -> str:
    src = os.path.join(CSRC, "rmat", "rmat.c")
    out = os.path.join(HERE, "librmat.so")
    tmp = out + ".tmp"
    _run(["gcc", "-std=c99", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", src, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


def build_csbfs(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(CSRC, "csbfs", "*.hip")))
    if not srcs:
        raise RuntimeError("no HIP sources found")
    out = os.path.join(HERE, "libcsbfs.so")
    tmp = out + ".tmp"
    _run([HIPCC, *HIP_FLAGS, *srcs, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


def build_all(verbose: bool = False) -> list[str]:
    return [build_rmat(verbose), build_csbfs(verbose)]


if __name__ == "__main__":
    for p in build_all(verbose=True):
        print(p)

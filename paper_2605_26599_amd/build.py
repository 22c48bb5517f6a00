"""Build libtde.so (gfx950 HIP kernels + C-ABI) in place with hipcc, and
libtde_host.so (the host CPU BR baseline) with g++."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtde.so")
ARCH = os.environ.get("TDE_OFFLOAD_ARCH", "gfx950")

SOURCES = ["tde_kernels.hip", "tde_api.cpp", "tde_planner.cpp", "tde_noalloc.hip", "tde_dense.hip"]

HIPCC_FLAGS = [
    "-O3",
    "-std=c++17",
    f"--offload-arch={ARCH}",
    "-fPIC",
    "-shared",
    # keep the compiler from emitting packed FP32 instructions on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


HOST_LIB = os.path.join(HERE, "libtde_host.so")
HOST_FLAGS = ["-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared"]


def build_host(verbose: bool = False) -> str:
    """libtde_host.so: the host CPU boundary-row D&C baseline (g++, OpenMP)."""
    cxx = os.environ.get("CXX", "g++")
    tmp = HOST_LIB + ".tmp"
    cmd = [cxx] + HOST_FLAGS + ["-o", tmp, os.path.join(CSRC, "host_br.cpp")]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("g++ failed building libtde_host.so")
    os.replace(tmp, HOST_LIB)
    return HOST_LIB


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libtde.so")
    os.replace(tmp, LIB)
    build_host(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

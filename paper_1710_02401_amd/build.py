"""Build the SWR HIP library (libswr.so) in-tree for gfx950.

The host geometry is compiled by g++ without floating-point contraction;
kernels and the C ABI by hipcc.  Object files go to _build/ next to this
file; the shared library is written next to this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libswr.so")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    geo = os.path.join(BUILD, "geometry.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-c",
          os.path.join(CSRC, "geometry.cpp"), "-o", geo], verbose)
    objs.append(geo)
    for src in ("kernels.hip", "wide.hip", "block.hip", "slater.hip", "capi.hip", "mlp.hip"):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        _run(["hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

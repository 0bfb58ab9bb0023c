"""Build libqwexp.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libqwexp.so")

SOURCES = ["qw_action.hip", "qw_batched.hip", "qw_grad.hip", "qw_cfet.hip", "qw_coeffs.cpp"]

# Packed fp32 instructions are disabled for all device code; the host pass of
# hipcc warns that it does not know the feature, which is harmless.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(bdir, src + ".o")
        cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-c", path, "-o", obj,
               "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-result"]
        if src.endswith(".hip"):
            cmd += DEVICE_FLAGS
        else:
            cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-c", path, "-o", obj, "-I", INCLUDE, "-I", CSRC, "-Wall"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

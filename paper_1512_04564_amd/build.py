"""Build libctrlalm.so (HIP, gfx950) in-tree with hipcc.

Every HIP source is compiled for gfx950 with packed-FP32 instructions disabled, then linked into one
shared library next to this file. ``build()`` always recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libctrlalm.so")
ARCH = os.environ.get("CTRLALM_ARCH", "gfx950")

# (source, extra flags). The projector / update kernels carry no NaN semantics; reductions keep them.
SOURCES = [("ct_geom.cpp", []), ("ct_kernels.hip", ["-fno-honor-nans"]), ("ct_reduce.hip", []), ("ct_fbp.hip", []),
           ("ct_unet.hip", []), ("ct_api.hip", []), ("ct_helix_tables.cpp", []), ("ct_helix.hip", [])]

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _hipcc() -> str:
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src, extra in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [_hipcc(), *HIPCC_FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

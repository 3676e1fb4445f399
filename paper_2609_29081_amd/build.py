"""Build the HIP library libaf.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaf.so")
# (source, object, extra flags): the 2D stage is compiled twice, as the FP64
# stage (16 x 7 tiles) and as the mixed-precision stage (FP32 stencils, whose
# smaller LDS footprint admits 16 x 10 tiles)
SOURCES = [("af_capi.cpp", "af_capi.o", []),
           ("af_common.hip", "af_common.o", []),
           ("af_kern1d.hip", "af_kern1d.o", []),
           ("af_stage2d.hip", "af_stage2d_fp64.o",
            ["-DAF_STAGE_REAL=double", "-DAF_STAGE_TY=7", "-DAF_STAGE_ENTRY=stage2d_fp64"]),
           ("af_stage2d.hip", "af_stage2d_mixed.o",
            ["-DAF_STAGE_REAL=float", "-DAF_STAGE_TY=10", "-DAF_STAGE_ENTRY=stage2d_mixed"])]
ARCH = "gfx950"


def hip_flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # no packed-FP32 instruction selection
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src, oname, extra in SOURCES:
        obj = os.path.join(bdir, oname)
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = ["hipcc", *hip_flags(), *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)

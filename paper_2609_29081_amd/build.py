"""Build the HIP library libaf.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaf.so")
# The 2D stage is compiled once per variant (arithmetic type, tile height):
# the FP64 stage with 16x7 tiles (the largest its LDS admits) and 16x5, the
# mixed-precision stage (FP32 stencils) with 16x14, 16x10 and 16x7.  The
# first variant of each precision is the one single-instance stages use; the
# batch autotuner chooses among all of a precision.  (entry name, type, TY)
STAGE_VARIANTS = [("stage2d_fp64_t7", "double", 7), ("stage2d_fp64_t5", "double", 5),
                  ("stage2d_mixed_t14", "float", 14), ("stage2d_mixed_t10", "float", 10),
                  ("stage2d_mixed_t7", "float", 7)]
# (source, object, extra flags)
SOURCES = [("af_capi.cpp", "af_capi.o", []),
           ("af_variants.cpp", "af_variants.o", ["--cuda-host-only"]),
           ("af_common.hip", "af_common.o", []),
           ("af_kern1d.hip", "af_kern1d.o", []),
           ("af_learn.hip", "af_learn.o", [])] + [
    ("af_stage2d.hip", f"{name}.o",
     [f"-DAF_STAGE_REAL={real}", f"-DAF_STAGE_TY={ty}", f"-DAF_STAGE_ENTRY={name}",
      # no hoisting of loop-invariant values out of the persistent tile
      # loop: held across all phases they spilled; recomputed, the FP64
      # stage spills nothing and runs 2 % faster
      "-mllvm", "--disable-machine-licm"])
    for name, real, ty in STAGE_VARIANTS]
ARCH = "gfx950"


def hip_flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # no packed-FP32 instruction selection
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # multiply-adds fused within one expression only: the rounding of
            # every result follows from the source, so that the template
            # instances of a kernel (single instance, batch, given blend)
            # round alike
            "-ffp-contract=on",
            # the backend's own register-pressure trackers in the scheduler:
            # the 2D stage spills half as much (32 bytes per lane) and runs
            # 5 % faster in FP64
            "-mllvm", "--amdgpu-use-amdgpu-trackers",
            "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for src, oname, extra in SOURCES:
        obj = os.path.join(bdir, oname)
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = ["hipcc", *hip_flags(), *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, p in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)

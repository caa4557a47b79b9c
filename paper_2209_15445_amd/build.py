"""Builds libems.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libems.so")
SOURCES = ["ems_kernels.hip", "ems_primaries.hip", "ems_static.hip", "ems_api.cpp", "ems_tables.cpp", "ems_server.cpp", "ems_geometry.cpp"]
# Compiled on its own with SLAB_F32_FLAGS, then linked with the rest: the
# mixed-form slab-stack kernels, scheduled for instruction-level parallelism
# (4% shorter mixed e-/e+ launches on the 10^5-event beam; the same setting
# made the FP64 and box-geometry kernels slower).
SLAB_F32_SOURCE = "ems_kernels_slab_f32.hip"
SLAB_F32_FLAGS = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",                     # native global FP64 atomic add
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-pthread",
]


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    obj = os.path.join(HERE, "ems_kernels_slab_f32.o")
    compile_only = [f for f in FLAGS if f != "-shared"]
    steps = [
        [HIPCC, *compile_only, *SLAB_F32_FLAGS, *extra, "-c", "-o", obj, os.path.join(CSRC, SLAB_F32_SOURCE)],
        [HIPCC, *FLAGS, *extra, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES] + ["-x", "none", obj],
    ]
    for cmd in steps:
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    os.remove(obj)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])

"""Build libbysdf.so (gfx950) in-tree with hipcc.

    python -m paper_2401_12724_amd.build

Every HIP source is compiled with packed-FP32 instruction selection turned
off (``-Xclang -target-feature -Xclang -packed-fp32-ops``).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbysdf.so")
SOURCES = ["bysdf_lib.hip", "yarn_scene.hip", "render.hip"]
HEADERS = ["bysdf_math.hpp", "bysdf_model.hpp", "bysdf_multi.hpp", "bysdf_opcount.hpp", "bysdf_dual.hpp",
           "yarn_tube.hpp", "yarn_build.hpp", "philox.hpp",
           "lib_internal.hpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP32 division and square root from the hardware reciprocal / root
    # (about 1 ulp); FP64 stays correctly rounded
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libbysdf.so (always recompiles)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + HIPCC_FLAGS + ["-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS]
    deps.append(os.path.join(ROOT, "include", "bysdf.h"))
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)

"""Build libbysdf.so (gfx950) in-tree with hipcc, and libbysdf_audit.so (the
host-side precision audit of the kernels' model, a measurement tool that
libbysdf does not link).

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
AUDIT_SOURCE = "precision_audit.hip"
AUDIT_LIB = os.path.join(HERE, "libbysdf_audit.so")
HEADERS = ["bysdf_math.hpp", "math_tables.inc", "bysdf_model.hpp", "bysdf_multi.hpp", "bysdf_opcount.hpp", "bysdf_dual.hpp",
           "yarn_tube.hpp", "yarn_build.hpp", "philox.hpp",
           "lib_internal.hpp", "bysdf_precision.hpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP32 division and square root from the hardware reciprocal / root
    # (about 1 ulp); FP64 stays correctly rounded
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libbysdf.so (always recompiles): one
    object per source, compiled in parallel, then linked."""
    tag = "%d" % os.getpid()
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".%s.o" % tag))
        cmd = ["hipcc"] + [f for f in HIPCC_FLAGS if f != "-shared"] + ["-c", "-o", obj,
                                                                        os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        objs.append(obj)
        procs.append(subprocess.Popen(cmd))
    audit_tmp = AUDIT_LIB + ".tmp" + tag
    cmd = ["hipcc"] + HIPCC_FLAGS + ["-o", audit_tmp, os.path.join(CSRC, AUDIT_SOURCE)]
    if verbose:
        print(" ".join(cmd), flush=True)
    procs.append(subprocess.Popen(cmd))
    rcs = [p.wait() for p in procs]
    try:
        if any(rcs):
            raise subprocess.CalledProcessError(max(rcs), "hipcc -c")
        tmp = LIB + ".tmp" + tag
        cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
        os.replace(audit_tmp, AUDIT_LIB)
    finally:
        if os.path.exists(audit_tmp):
            os.remove(audit_tmp)
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB) or not os.path.exists(AUDIT_LIB):
        return True
    t = min(os.path.getmtime(LIB), os.path.getmtime(AUDIT_LIB))
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS + [AUDIT_SOURCE]]
    deps.append(os.path.join(ROOT, "include", "bysdf.h"))
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)

"""Build libmxn.so (the HIP library behind include/mxn.h) for gfx950 in-tree.

    python -m paper_1306_1737_amd.build

Every HIP translation unit is compiled with packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops).  grid.hip, pairlist.hip and
rdf.hip are compiled with -ffp-contract=off because the sort keys, bounding
boxes, the pair-list predicate and the histogram bins are defined by
separately rounded FP32 operations (forces.hip writes its one such expression,
the gathers' image shift, with explicit round-to-nearest operations).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmxn.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("MXN_OFFLOAD_ARCH", "gfx950")

SOURCES = {
    "api.hip": [],
    "grid.hip": ["-ffp-contract=off"],
    "pairlist.hip": ["-ffp-contract=off"],
    "rdf.hip": ["-ffp-contract=off"],
    "forces.hip": [],
    "recount.hip": [],
    "mlp.hip": [],
    "buffer.cpp": [],
}
COMMON = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-Wall", "-Wno-unused-result"]


def _hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _compile(src, extra):
    obj = os.path.join(BUILD, src + ".o")
    lang = ["-x", "hip"]
    cmd = [_hipcc()] + lang + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), SOURCES.items()))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

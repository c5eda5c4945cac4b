"""Build step of libcorr.so: hipcc for gfx950, in-tree.

``python -m paper_1711_05075_amd.build`` or ``build_library()`` compiles the
kernels and the host side into ``paper_1711_05075_amd/libcorr.so``.  The build
needs no GPU (hipcc cross-compiles for gfx950).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcorr.so")
ARCH = "gfx950"

# packed FP32 instructions stay off: hipcc may otherwise form v_pk_* float ops
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]
# the correlation kernels contract no multiply-add on their own: their fused
# operations are written out, so results are bitwise the same for every launch
# shape the autotuner may pick
PER_FILE = {"corr_kernels.hip": ["-ffp-contract=off"], "raster_kernels.hip": ["-ffp-contract=off"]}


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n%s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return r


def build_library(verbose: bool = False) -> str:
    hipcc = _hipcc()
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs, cmds = [], []
    for src, lang in (("corr_kernels.hip", "hip"), ("raster_kernels.hip", "hip"), ("corr_host.cpp", "hip"),
                      ("prop_kernels.hip", "hip"), ("prop_host.cpp", "hip")):
        obj = os.path.join(bdir, src + ".o")
        cmds.append([hipcc, "-x", lang, "--offload-arch=" + ARCH, *COMMON, *DEVICE_FLAGS, *PER_FILE.get(src, []),
                     "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # the four translation units compile side by side
    with ThreadPoolExecutor(max_workers=len(cmds)) as pool:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        list(pool.map(_run, cmds))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))

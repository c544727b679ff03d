"""Build the selected-inversion shared library for gfx950 with hipcc.

Produces ``paper_1604_02528_amd/_lib/libselinv.so`` (the C ABI of
include/selinv.h).  Every HIP translation unit is compiled with the packed-FP32
feature switched off, the host parts with -march=x86-64-v3.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libselinv.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["symbolic.cpp", "factor_host.cpp", "tune.cpp", "capi.cpp", "kernels.hip", "adjoint.hip", "factor.hip"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return [
        "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-march=x86-64-v3", "-pthread",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    ]


def build(verbose=False, jobs=None):
    os.makedirs(OUT_DIR, exist_ok=True)
    cc = hipcc()
    objs = []
    cmds = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OUT_DIR, src.replace(".", "_") + ".o")
        objs.append(obj)
        cmd = [cc, *common_flags(), "-c", path, "-o", obj]
        if src.endswith(".cpp"):
            cmd = [cc, *common_flags(), "-x", "hip", "-c", path, "-o", obj]
        cmds.append(cmd)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return r.stderr

    with ThreadPoolExecutor(max_workers=jobs or min(len(cmds), 8)) as ex:
        for err in ex.map(run, cmds):
            if verbose and err.strip():
                print(err, file=sys.stderr)
    link = [cc, "-shared", "-fPIC", "--offload-arch=gfx950", "-pthread", "-o", LIB + ".tmp", *objs]
    run(link)
    os.replace(LIB + ".tmp", LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Builds libskm.so for gfx950 with hipcc (in-tree, under lib/)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "lib")
LIB = os.path.join(OUT, "libskm.so")
SOURCES = ["kernels_assign.hip", "kernels_update.hip", "kernels_dense.hip",
           "kernels_seed.hip", "skm_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # packed FP32 instructions stay off (hipcc flag for the device pass)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-Wno-pass-failed"]


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    objs = []

    def compile_one(name):
        src = os.path.join(SRC, name)
        obj = os.path.join(OUT, name.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, "-I", os.path.join(HERE, "..", "include"), "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        noise = "is not a recognized feature for this target"
        err = "\n".join(ln for ln in r.stderr.splitlines() if noise not in ln)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (name, err))
        if verbose and err.strip():
            print(err, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    r = subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

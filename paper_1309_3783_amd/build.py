"""Build the gfx950 HIP library libsphcell.so in-tree with hipcc.

Every source under csrc/ is compiled for gfx950 only, without fast-math and
with packed FP32 instructions disabled, then linked into one shared library
next to this file.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsphcell.so")
SOURCES = ["sph_prims.hip", "sph_build.hip", "sph_interact.hip", "sph_integrate.hip", "sph_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(HERE, "..", "include")]


def _compile(src: str, objdir: str) -> str:
    obj = os.path.join(objdir, src.replace(".hip", ".o"))
    subprocess.run([HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], check=True,
                   stdout=subprocess.PIPE, stderr=subprocess.PIPE)
    return obj


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        futs = [ex.submit(_compile, s, objdir) for s in SOURCES]
        objs = []
        for f in futs:
            try:
                objs.append(f.result())
            except subprocess.CalledProcessError as e:
                raise RuntimeError("hipcc failed:\n" + e.stderr.decode(errors="replace")) from None
    tmp = OUT + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], check=True)
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)

"""Builds libcomposite.so (HIP for gfx950) in the package directory, and
libceiling.so, the benchmark's same-traffic reference kernel.

Every HIP source is compiled with hipcc for gfx950 only; packed FP32
instructions are disabled in device code.  Objects go to a build folder
beside the sources; the shared library lands next to this file."""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libcomposite.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["kernels.hip", "context.hip", "batch.hip", "serve.hip", "verify.hip"]
CEILING_SRC = "ceiling.hip"
CEILING_OUT = os.path.join(PKG, "libceiling.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES) + 1)) as ex:
        objs = list(ex.map(_compile, SOURCES + [CEILING_SRC]))
    for out, parts in ((OUT, objs[:-1]), (CEILING_OUT, objs[-1:])):
        tmp = out + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *parts, "-lpthread"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link of {os.path.basename(out)} failed:\n{r.stderr}")
        os.replace(tmp, out)
        if verbose:
            print(f"built {out}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

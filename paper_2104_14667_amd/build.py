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
SOURCES = ["kernels.hip", "repack.hip", "utility.hip", "context.hip", "batch.hip", "serve.hip", "verify.hip", "noalloc.hip"]
CEILING_SRC = "ceiling.hip"
CEILING_OUT = os.path.join(PKG, "libceiling.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer: only the host
# pass is instrumented (device code is compiled as usual).  The result is a
# CPU test build of the same sources, loaded with the sanitizer runtime
# preloaded; nothing on the device path uses it.
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-g"]
SAN_DIR = os.path.join(BUILD, "hostsan")


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
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


def build_host_sanitized(verbose: bool = False) -> str:
    """libcomposite.so with ASan and UBSan in its host code, under
    _build/hostsan/ (run it with the clang ASan runtime preloaded)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, SAN_DIR, SAN_FLAGS), SOURCES))
    out = os.path.join(SAN_DIR, "libcomposite.so")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", out, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitized link failed:\n{r.stderr}")
    if verbose:
        print(f"built {out}")
    return out


def sanitizer_runtime() -> str:
    """Path of the clang ASan runtime that matches hipcc's compiler."""
    r = subprocess.run([os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin",
                        "clang"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isfile(path):
        raise RuntimeError("clang ASan runtime not found")
    return path


if __name__ == "__main__":
    if "--host-sanitize" in sys.argv:
        build_host_sanitized(verbose=True)
        sys.exit(0)
    build(verbose=True)
    sys.exit(0)

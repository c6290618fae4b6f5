"""Compile libsfm.so (HIP C++ for gfx950) in-tree.

Usage: python -m paper_1406_6923_amd.build_lib  (or build() from Python).
Every HIP source is compiled with packed-FP32 instructions disabled; the library links
only the HIP runtime (every kernel, the ROM build's FP64 products included, is in csrc/).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsfm.so")
ARCH = os.environ.get("SFM_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-result"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


# The debug preset: SFM_DEBUG launch checks (shapes and grids against what each kernel assumes,
# abort on violation), host code under AddressSanitizer and UndefinedBehaviorSanitizer (device code
# is not instrumented), -O1 -g.  Load it with the sanitizer runtime preloaded.
DEBUG = ["-O1", "-g", "-DSFM_DEBUG", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
         "-Xarch_host", "-fsanitize=undefined"]
OBJ_DEBUG = os.path.join(PKG, "_build_debug")
LIB_DEBUG = os.path.join(PKG, "libsfm_debug.so")


def _compile(src: str, verbose: bool, debug: bool = False) -> str:
    obj = os.path.join(OBJ_DEBUG if debug else OBJ, os.path.basename(src) + ".o")
    flags = [f for f in COMMON if f != "-O3"] + DEBUG if debug else COMMON
    cmd = [_hipcc(), *flags, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [_hipcc(), "-x", "hip", *flags, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    if verbose and res.stderr.strip():
        print(res.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False, debug: bool = False) -> str:
    """Compile every source under csrc/ and link libsfm.so (libsfm_debug.so with debug=True, the
    debug preset above); returns the library path."""
    os.makedirs(OBJ_DEBUG if debug else OBJ, exist_ok=True)
    lib = LIB_DEBUG if debug else LIB
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, debug), srcs))
    tmp = lib + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
           "-Wl,-rpath,/opt/rocm/lib"]
    if debug:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Compile libghn.so for gfx950 with hipcc (in-tree, so the library travels with the tree)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(PKG, "libghn.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["ghn_api.hip", "ghn_hostenv.hip", "ghn_arrays.hip", "ghn_build.hip", "ghn_predict.hip", "ghn_tree.hip", "ghn_group.hip", "ghn_batch.hip", "ghn_tune.hip", "ghn_measure.hip"]

# -ffp-contract=off: FP64 distances and bounds are evaluated exactly as written.
# -packed-fp32-ops off: no packed FP32 instructions are generated.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libghn.so.  Returns the library path."""
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# Host sanitizer build: the host-only sources (entry points, environment switches) are
# compiled for the host alone with AddressSanitizer and UBSan; every other object, kernels
# included, is the ordinary one.  The driver (tests/cpu/host_sanitize.cpp) is linked with
# clang's sanitizer runtimes, which the library's instrumented code resolves against.
HOST_ONLY_SOURCES = ["ghn_api.hip", "ghn_hostenv.hip"]
SAN_DIR = os.path.join(PKG, "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "libghn_hostsan.so")
SAN_EXE = os.path.join(SAN_DIR, "host_sanitize")
SAN_DRIVER = os.path.join(ROOT, "tests", "cpu", "host_sanitize.cpp")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
             "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined"]
CLANGXX = os.environ.get("GHN_CLANGXX", "/opt/rocm/llvm/bin/clang++")


def _run(cmd, what):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s failed:\n%s\n%s" % (what, " ".join(cmd), r.stderr))


def build_sanitized(verbose: bool = False) -> str:
    """The host sanitizer library and its driver (SAN_EXE).  Reuses the ordinary objects
    of build(), compiling any that are missing."""
    os.makedirs(SAN_DIR, exist_ok=True)
    san_obj = os.path.join(ROOT, "_build", "san")
    os.makedirs(san_obj, exist_ok=True)
    objs = []
    for src in SOURCES:
        if src in HOST_ONLY_SOURCES:
            obj = os.path.join(san_obj, src.replace(".hip", ".o"))
            _run([HIPCC, "--cuda-host-only", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall",
                  "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")] + SAN_FLAGS +
                 ["-c", os.path.join(CSRC, src), "-o", obj], "hipcc (host sanitizer) " + src)
        else:
            obj = os.path.join(OBJ, src.replace(".hip", ".o"))
            if not os.path.exists(obj):
                os.makedirs(OBJ, exist_ok=True)
                obj = _compile(src)
        objs.append(obj)
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", SAN_LIB] + objs, "link " + SAN_LIB)
    _run([CLANGXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
          "-I" + os.path.join(ROOT, "include"), SAN_DRIVER, "-o", SAN_EXE, "-L" + SAN_DIR, "-lghn_hostsan",
          "-Wl,-rpath,$ORIGIN", "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], "link " + SAN_EXE)
    if verbose:
        print("built", SAN_EXE)
    return SAN_EXE


if __name__ == "__main__":
    build(verbose=True)
    build_sanitized(verbose=True)

"""Build libfusedpr.so in-tree for gfx950 with hipcc.

Every HIP source is compiled with packed-FP32 instruction selection disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``); the host-only C++
sources go through the same driver.  The library lands next to this file as
``libfusedpr.so``; objects go to ``_build/`` (not part of the source tree).
``build_all`` also builds the test variant ``libfusedpr_naive.so`` (FP32 sums
without compensation).
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfusedpr.so")
ARCH = "gfx950"

SOURCES = ["error.cpp", "csr_build.cpp", "plan.hip", "sweep.hip", "batched.hip", "adjoint.hip", "probe.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _compile(src: str, extra: list[str]) -> str:
    path = os.path.join(CSRC, src)
    tag = ("." + hashlib.sha1(" ".join(extra).encode()).hexdigest()[:8]) if extra else ""
    obj = os.path.join(BUILD, src + tag + ".o")
    if src.endswith(".hip"):
        cmd = [hipcc(), *COMMON, *DEVICE, *extra, "-c", path, "-o", obj]
    else:
        cmd = [hipcc(), *COMMON, *extra, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(extra: list[str] | None = None, verbose: bool = False, out: str | None = None) -> str:
    """Compile and link; `extra` flags go to every compile, `out` overrides the
    library path (variants built for measurements)."""
    os.makedirs(BUILD, exist_ok=True)
    extra = list(extra or [])
    lib_path = out or LIB
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), srcs))
    tmp = lib_path + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, lib_path)
    if verbose:
        print("built", lib_path)
    return lib_path


NAIVE_LIB = os.path.join(HERE, "libfusedpr_naive.so")


def build_all(verbose: bool = False) -> None:
    """The library, and its test variant with uncompensated FP32 sums
    (FPR_NAIVE_SUM=1, libfusedpr_naive.so), which the precision tests compare
    against."""
    build(verbose=verbose)
    build(["-DFPR_NAIVE_SUM=1"], verbose=verbose, out=NAIVE_LIB)


if __name__ == "__main__":
    if sys.argv[1:]:
        build(sys.argv[1:], verbose=True)
    else:
        build_all(verbose=True)

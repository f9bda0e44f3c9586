"""Build the SparkCL hot-path library for gfx950.

Produces, next to this file:
  libsparkcl.so       -- the C-ABI library (HIP kernels + host runtime), built
                         with hipcc --offload-arch=gfx950;
  libsparkcl_host.so  -- the pure host logic (arena, admission, tuning cache)
                         behind a small C shim, built with g++, for CPU tests.

Every HIP translation unit is compiled with -ffp-contract=off (the maps are
the binary32 definition step by step) and with packed-FP32 instructions
disabled.  Run: python -m paper_1505_01120_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsparkcl.so")
HOST_LIB = os.path.join(HERE, "libsparkcl_host.so")
ARCH = "gfx950"

HIP_SOURCES = ["kernels.hip", "api.cpp", "serve.cpp", "autotune.cpp", "tuning.cpp"]
HOST_SOURCES = ["tuning.cpp", "hostlogic_capi.cpp"]

COMMON = ["-std=c++17", "-O3", "-fPIC", "-fvisibility=hidden", "-Wall", "-Wextra", "-Wno-unused-parameter",
          "-I", INCLUDE, "-I", CSRC]
HIP_FLAGS = ["--offload-arch=" + ARCH, "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: the SparkCL library needs ROCm to build")
    return p


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + os.path.basename(cmd[-1]))


def build(verbose: bool = False) -> str:
    """Compile every source and link both libraries (always rebuilds)."""
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    cc = hipcc()

    def compile_hip(src: str) -> str:
        obj = os.path.join(out_dir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([cc, *COMMON, *HIP_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_hip, HIP_SOURCES))
    tmp = LIB + ".tmp"
    _run([cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp, "-lpthread"])
    os.replace(tmp, LIB)

    tmp = HOST_LIB + ".tmp"
    _run(["g++", *COMMON, "-shared", *[os.path.join(CSRC, s) for s in HOST_SOURCES],
          "-o", tmp])
    os.replace(tmp, HOST_LIB)
    if verbose:
        print("built", LIB, "and", HOST_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)

"""Build steps for the native libraries (run on any host; hipcc cross-compiles gfx950).

libmcm.so      the matching library: HIP kernels + host driver + C ABI
libmcmgen.so   the seeded input generators (plain C)
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN_LIB = os.path.join(HERE, "libmcmgen.so")
MCM_LIB = os.path.join(HERE, "libmcm.so")
BUILD_DIR = os.path.join(ROOT, "_build")

HIP_SOURCES = ["mcm_kernels.hip", "mcm_noalloc.hip"]
HOST_SOURCES = ["mcm_api.cpp", "mcm_batch.cpp", "mcm_server.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# gfx950 only; packed-FP32 instructions are disabled for every HIP object.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-fno-strict-aliasing",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _run(cmd, out):
    tmp = out + ".tmp"
    subprocess.run(cmd + ["-o", tmp], check=True)
    os.replace(tmp, out)
    return out


def build_gen() -> str:
    """Input generators: plain C with OpenMP, portable -O3 (no -march=native:
    the library travels to other hosts)."""
    return _run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                 os.path.join(CSRC, "graphgen.c"), "-lm"], GEN_LIB)


def build_mcm(verbose: bool = False) -> str:
    """Compile every HIP and host source for gfx950 and link libmcm.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src in HIP_SOURCES + HOST_SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src)]
        if verbose:
            cmd += ["-Rpass-analysis=kernel-resource-usage"]
        _run(cmd, obj)
        objs.append(obj)
    return _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs, MCM_LIB)


def build_all() -> None:
    build_gen()
    build_mcm()

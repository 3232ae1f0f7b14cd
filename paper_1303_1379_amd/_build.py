"""Build steps for the native libraries (run on any host; hipcc cross-compiles gfx950)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
GEN_LIB = os.path.join(HERE, "libmcmgen.so")


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


def build_all() -> None:
    build_gen()

"""Build steps for the native parts of the package (in-tree, for gfx950).

* ``libcsel.so``            -- the C-ABI library: HIP kernels + host entry points
                               (hipcc, --offload-arch=gfx950)
* ``inputs/libcsel_geometry.so`` -- host kd-tree helpers for the seeded inputs (gcc)

Every call recompiles.  ``python -m paper_2307_11648_amd.build`` runs both.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcsel.so")
GEO_SRC = os.path.join(PKG, "inputs", "geometry.c")
GEO_LIB = os.path.join(PKG, "inputs", "libcsel_geometry.so")

HIP_SOURCES = ["abi.cpp", "select.hip", "aggregate.hip", "apply.hip", "mlp.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-ffp-contract=fast",
    "-Wno-unused-command-line-argument",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r.stdout


def build_geometry() -> str:
    _run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", GEO_LIB, GEO_SRC, "-lm"])
    return GEO_LIB


def hip_sources():
    return [os.path.join(CSRC, s) for s in HIP_SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build_hip(extra_flags=None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + (extra_flags or []) + ["-I", INCLUDE, "-I", CSRC, "-o", tmp] + hip_sources()
    _run(cmd)
    os.replace(tmp, LIB)
    return LIB


def build_all() -> None:
    build_geometry()
    build_hip()


if __name__ == "__main__":
    build_all()
    print("built", LIB, GEO_LIB)

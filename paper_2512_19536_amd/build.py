"""Build libpdg.so (host C++ setup + HIP kernels for gfx950) in-tree.

Usage: ``python -m paper_2512_19536_amd.build`` or ``build()`` from Python.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpdg.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for every HIP compilation unit.
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          "-Wno-unused-result"]
HOST_ONLY = ["-mavx2", "-mfma", "-I/opt/rocm/include"]

SOURCES = [
    ("kernels.hip", "device"),
    ("mlp.hip", "device"),
    ("mlp_api.cpp", "host"),
    ("fem.cpp", "host"),
    ("schwarz_setup.cpp", "host"),
    ("api.cpp", "host"),
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src, kind in SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        path = os.path.join(CSRC, src)
        if kind == "device":
            cmd = [HIPCC] + DEVICE_FLAGS + COMMON + ["-c", path, "-o", obj]
        else:
            cmd = [HIPCC, "-x", "c++"] + COMMON + HOST_ONLY + ["-D__HIP_PLATFORM_AMD__", "-c", path, "-o", obj]
        _run(cmd, verbose)
        objs.append(obj)
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-o", tmp] + objs + ["-lpthread"], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))

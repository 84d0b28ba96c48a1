"""Build the in-tree shared library libbidomain.so for gfx950.

Host C++ (assembly, AMG setup) is compiled with g++ and OpenMP; the HIP translation unit with
hipcc for gfx950 only.  Packed FP32 instructions are disabled for every HIP object.
Usage:  python -m paper_2311_13914_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbidomain.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HOST_SOURCES = ["host_assemble.cpp", "host_ellipsoid.cpp", "host_amg.cpp"]
HIP_SOURCES = ["device.hip"]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:3])} ...")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["g++", "-O3", "-fPIC", "-fopenmp", "-std=c++17", "-Wall", *inc, "-c",
              os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", "-o", tmp, *objs, f"-L{ROCM}/lib", "-lamdhip64", "-fopenmp",
          f"-Wl,-rpath,{ROCM}/lib"], verbose)
    os.replace(tmp, LIB)
    return LIB


HOST_CHECK = os.path.join(BUILD, "host_check_asan")


def build_host_check(verbose: bool = False) -> str:
    """The host setup code (assembly, AMG setup) with its self-check driver, built with
    AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only; no HIP source)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [os.path.join(CSRC, f) for f in ["host_check.cpp"] + HOST_SOURCES]
    _run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fopenmp", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          *srcs, "-o", HOST_CHECK], verbose)
    return HOST_CHECK


if __name__ == "__main__":
    if "--host-check" in sys.argv:
        print(build_host_check(verbose=True))
    else:
        print(build(verbose=True))

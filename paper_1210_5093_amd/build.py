"""Build ``libdfaspec.so`` (HIP, gfx950 only) in-tree with hipcc, and the
host multicore matcher ``libdfahost.so`` with the host C++ compiler."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdfaspec.so")
PROBE = os.path.join(HERE, "lds_peak_probe")
HOST_LIB = os.path.join(HERE, "libdfahost.so")
CXX = os.environ.get("CXX", "g++")
SOURCES = ["dfa_compile.cpp", "dfa_api.cpp", "dfa_kernels.hip", "dfa_match2.hip",
           "dfa_batch.hip", "dfa_batch2.hip", "dfa_server.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions stay disabled in all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(HERE, "csrc", src)
        obj = os.path.join(objdir, src + ".o")
        cmd = [HIPCC, *COMMON, *DEVICE_FLAGS, "-x", "hip", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", *DEVICE_FLAGS, "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # measurement program for the LDS-lookup roofline denominator
    probe_src = os.path.join(HERE, "csrc", "lds_peak_probe.hip")
    cmd = [HIPCC, "-O3", "-std=c++17", *DEVICE_FLAGS, "-o", PROBE + ".tmp", probe_src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(PROBE + ".tmp", PROBE)
    build_host(verbose)
    return LIB


def build_host(verbose: bool = False) -> str:
    src = os.path.join(HERE, "csrc", "host_spec.cpp")
    cmd = [CXX, "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall",
           "-I", os.path.join(ROOT, "include"), "-o", HOST_LIB + ".tmp", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(HOST_LIB + ".tmp", HOST_LIB)
    return HOST_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

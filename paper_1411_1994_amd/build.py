"""Build the gfx950 shared library ``paper_1411_1994_amd/lib/liblsum.so`` with hipcc.

Every HIP/C++ source under ``csrc/`` is compiled for gfx950 only and linked into one shared
library exposing the C ABI of ``include/lsum.h``.  Run ``python paper_1411_1994_amd/build.py``
(as a script: importing the package would load the previous library).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(ROOT, "_build", "obj")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "liblsum.so")

SOURCES = ["lsum_host.cpp", "lsum_sinc_error.cpp", "lsum_tune.cpp", "lsum_runtime.cpp", "lsum_pipeline.cpp", "lsum_capi.cpp",
           "lsum_blas.cpp",
           "kernels_lattice.hip", "kernels_gemm.hip", "kernels_jacobi.hip", "scratch_noalloc.hip"]

# Packed FP32 instructions are disabled for all device code (only hand-checked FP32 paths).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found")
    return path


def compile_one(src: str) -> str:
    os.makedirs(OBJ, exist_ok=True)
    obj = os.path.join(OBJ, src + ".o")
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
           "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
    cmd += DEVICE_FLAGS
    if src == "lsum_host.cpp":
        cmd += ["-ffp-contract=off"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    noisy = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if noisy:
        sys.stderr.write(f"[{src}]\n" + "\n".join(noisy) + "\n")
    return obj


def build(verbose: bool = True) -> str:
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lrocblas", "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# The host-side steps (quadrature, snapping, lattice classes, request plans, the autotuner's
# file) with a self-test driver, compiled by the host compiler with AddressSanitizer and
# UndefinedBehaviorSanitizer: host code only, nothing for the GPU.
HOST_SELFTEST_SOURCES = ["host_selftest.cpp", "lsum_host.cpp", "lsum_sinc_error.cpp", "lsum_tune.cpp"]
HOST_SELFTEST = os.path.join(ROOT, "_build", "host_selftest")


def build_host_selftest(verbose: bool = True) -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    os.makedirs(os.path.dirname(HOST_SELFTEST), exist_ok=True)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(rocm, "include"), "-I", INCLUDE, "-I", CSRC]
    cmd += [os.path.join(CSRC, s) for s in HOST_SELFTEST_SOURCES]
    cmd += ["-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib"),
            "-o", HOST_SELFTEST]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"host self-test build failed\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    if verbose:
        print(f"built {HOST_SELFTEST}")
    return HOST_SELFTEST


if __name__ == "__main__":
    if "--host-selftest" in sys.argv:
        build_host_selftest()
    else:
        build()

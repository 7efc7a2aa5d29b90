"""Build libnpfem.so (C ABI + HIP kernels for gfx950) in-tree with hipcc.

Usage: python -m paper_1911_03062_amd.build_lib   (or build() from Python)
Object files go to paper_1911_03062_amd/_build/, the library to paper_1911_03062_amd/.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnpfem.so")
CHECK_LIB = os.path.join(HERE, "libnpfem_elemcheck.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["setup.cpp", "capi.cpp", "kernels_plain.hip", "kernels_fused.hip", "kernels_filter.hip",
           "kernels_contacts.hip", "kernels_global.hip"]

# Device code is compiled without packed-FP32 instructions (v_pk_*_f32).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Wall",
          "-Wno-unused-function", "-Wno-unused-variable", "-I", os.path.join(HERE, "..", "include")]


# The median filter's min/max need no NaN canonicalisation of their loaded inputs (NaN forces
# give unspecified filtered values, as IEEE min/max already drop NaNs).
FILE_FLAGS = {"kernels_filter.hip": ["-fno-honor-nans"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    cmd = [HIPCC, *COMMON, *DEVICE_FLAGS, *FILE_FLAGS.get(src, []), "-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *COMMON, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    # host build of the element math for CPU checks
    tmp = CHECK_LIB + ".tmp"
    cmd = [HIPCC, *COMMON, "-shared", "-o", tmp, os.path.join(CSRC, "elemcheck.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, CHECK_LIB)
    if verbose:
        print("built", LIB, "and", CHECK_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

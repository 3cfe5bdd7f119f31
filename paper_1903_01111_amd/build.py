"""Builds the HIP library paper_1903_01111_amd/liblbm_vibb.so for gfx950.

Kernels (.hip) are compiled by hipcc for gfx950; the host runtime and the
geometry (.cpp) by g++ against the HIP runtime headers; hipcc links them.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "liblbm_vibb.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

# (source, extra flags, object tag): the step kernels are compiled once per storage
# format (LBM_ST), so that the formats build in parallel
STORAGE_FORMATS = (0, 1, 2, 3, 4, 5)
HIP_UNITS = [("lbm_kernels.hip", [f"-DLBM_ST={k}"], f"st{k}") for k in STORAGE_FORMATS] + [
    ("lbm_adjoint.hip", [], ""), ("lbm_noalloc.hip", [], "")]
CXX_SOURCES = ["lbm_runtime.cpp", "lbm_batch.cpp", "lbm_geometry.cpp", "lbm_adjoint.cpp", "lbm_dispatch.cpp"]
HIP_SOURCES = sorted({u[0] for u in HIP_UNITS})

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               # packed FP32 instructions are kept out of the generated code
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               # multiply-adds fused within a source expression only: every kernel
               # instantiation (launch shape, rows per wavefront, batch) then rounds
               # the same way, which keeps their results bitwise equal
               "-ffp-contract=on",
               "-Wall", "-Wno-unused-function"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__"]


def _inc():
    return ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", os.path.join(ROCM, "include")]


def _compile(unit, verbose):
    src, extra, tag = unit if isinstance(unit, tuple) else (unit, [], "")
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + (f".{tag}" if tag else "") + ".o")
    if src.endswith(".hip"):
        cmd = [os.path.join(ROCM, "bin", "hipcc"), *HIPCC_FLAGS, *extra, *_inc(), "-c", path, "-o", obj]
    else:
        cmd = ["g++", *CXX_FLAGS, *_inc(), "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = HIP_UNITS + CXX_SOURCES
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [os.path.join(ROCM, "bin", "hipcc"), "--offload-arch=gfx950", "-shared", "-fPIC",
           "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def sources():
    headers = sorted(os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h"))
    return [os.path.join(CSRC, s) for s in HIP_SOURCES + CXX_SOURCES] + headers + [
        os.path.join(ROOT, "include", "lbm.h")]


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in sources())


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

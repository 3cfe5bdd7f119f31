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
# host code with AddressSanitizer and UndefinedBehaviorSanitizer (g++; the HIP
# objects are the ordinary ones): loaded instead of LIB when LBM_SANITIZE is set
LIB_SAN = os.path.join(HERE, "liblbm_vibb_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]
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


def _compile(unit, verbose, sanitize=False):
    src, extra, tag = unit if isinstance(unit, tuple) else (unit, [], "")
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + (f".{tag}" if tag else "") + ".o")
    if src.endswith(".hip"):
        cmd = [os.path.join(ROCM, "bin", "hipcc"), *HIPCC_FLAGS, *extra, *_inc(), "-c", path, "-o", obj]
    elif sanitize:
        obj = os.path.join(BUILD, src + ".san.o")
        cmd = ["g++", *CXX_FLAGS, *SAN_FLAGS, *_inc(), "-c", path, "-o", obj]
    else:
        cmd = ["g++", *CXX_FLAGS, *_inc(), "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build_sanitized(verbose: bool = False) -> str:
    """LIB_SAN: the HIP objects of the ordinary build with the host sources
    compiled by g++ under AddressSanitizer and UBSan, linked by g++ against the HIP
    runtime (run the CPU tests with LBM_SANITIZE=1 and the sanitizer runtimes
    preloaded)."""
    os.makedirs(BUILD, exist_ok=True)
    hip_objs = [os.path.join(BUILD, u[0] + (f".{u[2]}" if u[2] else "") + ".o") for u in HIP_UNITS]
    if any(not os.path.exists(o) for o in hip_objs):
        build(verbose)
    with ThreadPoolExecutor(max_workers=min(8, len(CXX_SOURCES))) as ex:
        san_objs = list(ex.map(lambda s: _compile(s, verbose, sanitize=True), CXX_SOURCES))
    tmp = LIB_SAN + ".tmp"
    cmd = ["g++", "-shared", "-fPIC", *SAN_FLAGS, "-o", tmp, *hip_objs, *san_objs,
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_SAN)
    return LIB_SAN


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
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))

"""Compiles the FP64 CPU oracle (test infrastructure only) into oracle/liblbm_oracle.so.

The oracle source is compiled twice, once on double and once on double _Complex
(complex-step derivatives), and linked into one shared object.  Strict IEEE
FP64: no FMA contraction, no fast-math.  A second library,
oracle/liblbm_oracle_omp.so, is the same source built with OpenMP (its per-node
loops run over rows on several threads); it times the oracle on all host cores
and runs the oracle on full-size workloads, and gives bitwise the serial results.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")
LIB_OMP = os.path.join(HERE, "liblbm_oracle_omp.so")
# both builds under AddressSanitizer and UBSan, loaded instead of LIB and LIB_OMP
# when LBM_SANITIZE is set (CPU tests only)
LIB_SAN = os.path.join(HERE, "liblbm_oracle_san.so")
LIB_SAN_OMP = os.path.join(HERE, "liblbm_oracle_omp_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall"]


def _build_one(lib, omp, verbose, san=False):
    objs = []
    flags = CFLAGS + (["-fopenmp"] if omp else []) + (SAN_FLAGS if san else [])
    for tag, extra in (("real", []), ("cplx", ["-DORC_COMPLEX"])):
        obj = os.path.join(HERE, f"_lbm_oracle_{tag}{'_omp' if omp else ''}{'_san' if san else ''}.o")
        cmd = ["gcc", *flags, *extra, "-c", SRC, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = ["gcc", "-shared", *(["-fopenmp"] if omp else []), *(SAN_FLAGS if san else []), "-o", tmp, *objs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


def build(verbose: bool = False) -> str:
    _build_one(LIB_OMP, True, verbose)
    return _build_one(LIB, False, verbose)


def build_sanitized(verbose: bool = False) -> str:
    _build_one(LIB_SAN_OMP, True, verbose, san=True)
    return _build_one(LIB_SAN, False, verbose, san=True)


def ensure_built(omp: bool = False) -> str:
    """Builds only if the library is missing or older than its source (the
    sanitized builds with LBM_SANITIZE set)."""
    if os.environ.get("LBM_SANITIZE"):
        lib = LIB_SAN_OMP if omp else LIB_SAN
        if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
            build_sanitized()
        return lib
    lib = LIB_OMP if omp else LIB
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
        build()
    return lib


if __name__ == "__main__":
    print(build_sanitized(verbose="-v" in sys.argv) if "--sanitize" in sys.argv else build(verbose="-v" in sys.argv))

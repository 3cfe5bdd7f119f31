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

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall"]


def _build_one(lib, omp, verbose):
    objs = []
    flags = CFLAGS + (["-fopenmp"] if omp else [])
    for tag, extra in (("real", []), ("cplx", ["-DORC_COMPLEX"])):
        obj = os.path.join(HERE, f"_lbm_oracle_{tag}{'_omp' if omp else ''}.o")
        cmd = ["gcc", *flags, *extra, "-c", SRC, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = ["gcc", "-shared", *(["-fopenmp"] if omp else []), "-o", tmp, *objs, "-lm"]
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


def ensure_built(omp: bool = False) -> str:
    """Builds only if the library is missing or older than its source."""
    lib = LIB_OMP if omp else LIB
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
        build()
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

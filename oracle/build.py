"""Compiles the FP64 CPU oracle (test infrastructure only) into oracle/liblbm_oracle.so.

The oracle source is compiled twice, once on double and once on double _Complex
(complex-step derivatives), and linked into one shared object.  Strict IEEE
FP64: no FMA contraction, no fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall"]


def build(verbose: bool = False) -> str:
    objs = []
    for tag, extra in (("real", []), ("cplx", ["-DORC_COMPLEX"])):
        obj = os.path.join(HERE, f"_lbm_oracle_{tag}.o")
        cmd = ["gcc", *CFLAGS, *extra, "-c", SRC, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-shared", "-o", tmp, *objs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


def ensure_built() -> str:
    """Builds only if the library is missing or older than its source."""
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

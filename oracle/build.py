"""Compile the oracle's C sources (test infrastructure only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "sweep.c"), os.path.join(HERE, "spectral.c")]
LIB = os.path.join(HERE, "_oracle_sweep.so")


def build(force: bool = True) -> str:
    """Build oracle/_oracle_sweep.so with gcc (-O2, OpenMP, no FP contraction)."""
    stale = not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(s) for s in SRCS)
    if force or stale:
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-std=c11", *SRCS, "-lm", "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

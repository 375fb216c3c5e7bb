"""Compile the oracle's C sweep (test infrastructure only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sweep.c")
LIB = os.path.join(HERE, "_oracle_sweep.so")


def build(force: bool = True) -> str:
    """Build oracle/_oracle_sweep.so with gcc (-O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-std=c11", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

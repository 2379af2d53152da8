"""Build the CPU FP64 oracle shared library (test infrastructure).

gcc, FP64, no contraction of multiply-adds so that every operation rounds as
written; OpenMP over the outer loops only (the arithmetic of a cell does not
depend on the thread count).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle_eos.c", "oracle_scheme.c", "oracle_field.c", "oracle_baro.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-function", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def needs_build():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = SOURCES + ["oracle.h", "oracle_internal.h"]
    return any(os.path.getmtime(os.path.join(HERE, s)) > t for s in deps)


if __name__ == "__main__":
    print(build(verbose=True))

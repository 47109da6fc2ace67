"""Compile the C part of the oracle (test infrastructure) into oracle/_build/."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
SRC = os.path.join(HERE, "raster.c")
LIB = os.path.join(OUT_DIR, "liboracle_raster.so")
SRC_RVQ = os.path.join(HERE, "rvq.c")
LIB_RVQ = os.path.join(OUT_DIR, "liboracle_rvq.so")


def _cc(src, lib, verbose, openmp=True):
    os.makedirs(OUT_DIR, exist_ok=True)
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math"] + (["-fopenmp"] if openmp else []) + \
          ["-shared", "-fPIC", "-Wall", "-Wno-unused-variable", src, "-o", lib + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def build(verbose=False):
    _cc(SRC_RVQ, LIB_RVQ, verbose, openmp=False)
    return _cc(SRC, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))

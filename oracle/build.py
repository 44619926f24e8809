"""Compile the oracle shared library with gcc (plain C, FP64, OpenMP).

``-ffp-contract=off`` keeps every multiply and add separately rounded, so the
oracle's arithmetic is the one written in the source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["lbm_ref.c", "mlp_ref.c", "forest_ref.c"]
LIB = os.path.join(HERE, "liblbm_ref.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c11",
           "-Wall", "-Wextra", "-shared", "-fPIC"]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    cmd += ["-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

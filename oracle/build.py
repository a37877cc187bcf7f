"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so.

Flags: no contraction of a*b+c into fma, no fast-math, x86-64-v3 (hardware fma
for the explicit fma() calls; runs on any AVX2 host), OpenMP across pairs.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-march=x86-64-v3", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

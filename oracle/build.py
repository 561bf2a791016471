"""Build the oracle's shared library (plain C, gcc, OpenMP over partitions).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use the oracle.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lrspike_oracle.c")
LIB = os.path.join(HERE, "liblrspike_oracle.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-Wno-unknown-pragmas", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

"""Build the CPU oracle shared library (test infrastructure only).

gcc, -O2, no fused multiply-add (-ffp-contract=off) and no fast-math, so
every floating-point operation happens in the order the source writes it.
OpenMP parallelises only over independent walkers between sync points;
results do not depend on the thread count.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rewl_oracle.c")
LIB = os.path.join(HERE, "liboracle_rewl.so")


def build(force=True):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

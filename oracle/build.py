"""Build the CPU oracle library (test infrastructure only).

Compiles ``cmo.c`` with gcc into ``libcmoracle.so`` next to this file:
strict IEEE arithmetic (no fast-math, no FMA contraction), OpenMP over runs.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libcmoracle.so")
SRC = os.path.join(HERE, "cmo.c")

CFLAGS = ["-O3", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
          "-fPIC", "-shared", "-march=x86-64-v2", "-Wall", "-Wextra", "-Werror"]


def build(force=True):
    """Compile the oracle; with force=False only when the library is missing."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

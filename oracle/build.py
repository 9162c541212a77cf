"""Compile the FP64 oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, no fast-math, OpenMP over batch rows.  Called by
``__graft_entry__.build()`` and, when the library is missing, by the oracle
loader itself.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fft_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(out=LIB, src=SRC, extra=()):
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
           *extra, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build())
    sys.exit(0)

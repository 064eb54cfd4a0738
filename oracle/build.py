"""Build the CPU oracle library (test infrastructure only).

    python oracle/build.py

compiles oracle/dqref.c with gcc into oracle/libdqref.so. IEEE semantics are
kept strict: no fast-math, no floating-point contraction.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libdqref.so")


def build(verbose=False):
    src = os.path.join(HERE, "dqref.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
           "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

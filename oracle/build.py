"""Build the CPU oracle library (test infrastructure; never loaded by the
product path).  Plain C, IEEE binary64, no contraction, no fast-math."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")

FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
         "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "orc.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", *FLAGS, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

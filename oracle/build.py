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


SRC = os.path.join(HERE, "orc.c")


def build(verbose: bool = False, src: str = SRC, out: str = LIB) -> str:
    """Compile `src` (the oracle's source, or a test's edited copy of it)
    into the shared library `out`."""
    tmp = out + ".tmp"
    cmd = ["gcc", *FLAGS, "-I", HERE, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

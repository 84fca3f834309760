"""Compile the C++ oracle into oracle/liboracle.so (g++, FP64, no FMA contraction).

Test infrastructure: the product library never links this.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
        "-Wall", "-Wextra", "-shared", "-fPIC", "-o", LIB + ".tmp", SRC, "-lpthread",
    ]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build step for the CPU oracle library (plain g++, no device code)."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "burgers_oracle.cpp")


def library_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Compile burgers_oracle.cpp with contraction off, so every expression rounds as written."""
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c++17", "-shared", "-fPIC",
           "-Wall", "-o", tmp, SOURCE]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

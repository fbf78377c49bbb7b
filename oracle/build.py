"""Build step of the CPU oracle: gcc, FP64, no fast-math, no FMA contraction,
OpenMP over z planes for the per-site loops (volume sums stay serial)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lattice_oracle.c")


def library_path() -> str:
    return os.path.join(HERE, "liblattice_oracle.so")


def build() -> str:
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())

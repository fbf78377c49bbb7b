"""Build the HIP library (gfx950) in-tree: paper_2102_01031_amd/csrc/liblattice.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, "lattice.hip")]
LIB = os.path.join(CSRC, "liblattice.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def library_path() -> str:
    return LIB


LIBS = ["-L/opt/rocm/lib", "-lhipfft"]   # power spectra: the library FFT


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, *SOURCES, *LIBS]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


CEILING_SRC = os.path.join(CSRC, "ceiling.hip")
CEILING = os.path.join(CSRC, "ceiling")


def build_ceiling(verbose: bool = False) -> str:
    """The streaming-bandwidth probe (an executable; see csrc/ceiling.hip)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [hipcc, *flags, "-o", CEILING + ".tmp", CEILING_SRC]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(CEILING + ".tmp", CEILING)
    return CEILING


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_ceiling(verbose=True))

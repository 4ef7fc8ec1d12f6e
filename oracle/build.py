"""Build the CPU oracle shared library (test infrastructure only).

The oracle is plain C++17 compiled with g++ and OpenMP (the step and its pins in
gmhc_oracle.cpp, the forward-mode derivatives of a 1D run in gmhc_tangent.cpp).  It shares no source with
the GPU library.  ``python oracle/build.py`` writes ``oracle/libgmhc_oracle.so``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "gmhc_oracle.cpp"), os.path.join(HERE, "gmhc_tangent.cpp")]
OUT = os.path.join(HERE, "libgmhc_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", OUT + ".tmp"] + SRC
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)

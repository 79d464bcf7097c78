"""Build the CPU oracle (test infrastructure) as ``oracle/liboracle.so``.

Plain g++, FP contraction off so that every rounding is the one written in
the source.  Run ``python oracle/build.py`` or call :func:`build`.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["philox.cpp", "genz.cpp", "special.cpp", "vegas.cpp", "cuhre.cpp", "suave.cpp", "divonne.cpp"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

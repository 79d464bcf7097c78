"""Build the CPU oracle (test infrastructure) as ``oracle/liboracle.so``.

Plain g++, FP contraction off so that every rounding is the one written in
the source.  Run ``python oracle/build.py`` or call :func:`build`.

``build(sanitize=True)`` (``python oracle/build.py --sanitize``) builds the
same sources with AddressSanitizer and UndefinedBehaviorSanitizer into
``oracle/liboracle_san.so``; ``oracle/sanitize.py`` runs the CPU test suite
against it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["philox.cpp", "genz.cpp", "special.cpp", "vegas.cpp", "cuhre.cpp", "suave.cpp", "divonne.cpp"]
LIB = os.path.join(HERE, "liboracle.so")
SAN_LIB = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]


def build(verbose=False, sanitize=False):
    out = SAN_LIB if sanitize else LIB
    cmd = ["g++", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra"]
    cmd += SAN_FLAGS if sanitize else ["-O2"]
    cmd += ["-o", out + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))

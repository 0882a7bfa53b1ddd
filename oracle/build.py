"""Build the C++ oracle (test infrastructure) into oracle/liboracle.so.

Plain g++, -O2 with floating-point contraction off so every product and sum is
rounded as written; OpenMP only parallelises loops whose results do not depend
on the thread count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qec_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fcx-limited-range",
        "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
        SRC, "-o", LIB + ".tmp",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build the FP64 CPU oracle (test infrastructure only) into oracle/libtgv_oracle.so.

Plain g++ with OpenMP, -O2 and -ffp-contract=off so that no multiply-add is
contracted: the oracle's rounding follows its source text.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tgv_oracle.cpp")
LIB = os.path.join(HERE, "libtgv_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

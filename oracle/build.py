"""Build the serial FP64 oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, -O3 -ffp-contract=off, no fast-math: the oracle's arithmetic is
evaluated exactly as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
FLAGS = ["-std=c11", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose=False):
    src = os.path.join(HERE, "su2_oracle.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc"] + FLAGS + ["-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the C oracle into ``oracle/libfporacle.so`` (test infrastructure only).

Plain gcc, -O2, no fast-math and no floating-point contraction, so every product and
sum is a separately rounded IEEE double operation; OpenMP for the loops whose outputs
belong to one iteration each (results independent of the thread count).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libfporacle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "fp_oracle.c")
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

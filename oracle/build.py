"""Builds the serial CPU oracle (test infrastructure) into oracle/libkmco.so.

Plain gcc, no GPU, no shared sources with the HIP library.  -ffp-contract=off
keeps every floating-point sum and product rounded as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libkmco.so")


def build(verbose=False):
    src = os.path.join(HERE, "kmco.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

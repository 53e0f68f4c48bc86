"""Build the sequential CPU oracle (``libixoracle.so``) with gcc.

Test infrastructure only: the oracle is compiled so that the tests, the smoke
check and the benchmark's CPU-baseline leg can call it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ixoracle.c")
LIB = os.path.join(HERE, "libixoracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

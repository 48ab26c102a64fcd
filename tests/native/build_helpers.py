"""Build the C helpers of the tests (plain gcc, OpenMP) in place."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsegment_reach.so")


def build():
    src = os.path.join(HERE, "segment_reach.c")
    subprocess.run(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", src, "-o", LIB + ".tmp"], check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())

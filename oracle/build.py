"""Build the CPU oracle's shared library (test infrastructure only).

The oracle is plain C compiled with gcc; it has no GPU code and shares no
source with the product library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "pa_oracle.c"), os.path.join(HERE, "toeplitz.c")]
LIB = os.path.join(HERE, "libpa_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-pthread", *SRCS, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)

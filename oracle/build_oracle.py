"""Compile the oracle's C part (joseph.c -> libjoseph_oracle.so) with gcc.

Test infrastructure: the library is loaded only by oracle/holo_oracle.py.
Built for the generic x86-64 target (the machine that runs the checks may
differ from the one that builds), without fast-math, so the double-precision
arithmetic is IEEE as written."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "joseph.c")
LIB = os.path.join(HERE, "libjoseph_oracle.so")


def build(verbose=True):
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-Wextra",
           "-o", tmp, SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle build failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)

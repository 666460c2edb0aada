"""Compile the CPU oracle into oracle/liboracle.so (test infrastructure).

build() makes the portable library the tests load.  build(native=True) makes
oracle/liboracle_native.so for the host it runs on (-march=native), which the
benchmark's CPU baseline times; both give bit-identical results (no
contraction, no fast-math: vectorisation cannot reorder the binary32 or
binary64 arithmetic)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_NATIVE = os.path.join(HERE, "liboracle_native.so")
# no contraction and no fast-math: binary32 results must follow the source order
FLAGS = ["-O3", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
         "-shared", "-Wall", "-Wno-unknown-pragmas"]


def build(verbose=False, native=False, out=None):
    lib = out or (LIB_NATIVE if native else LIB)
    cmd = ["gcc", *FLAGS, *(["-march=native"] if native else []), "-o", lib + ".tmp",
           os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, native="--native" in sys.argv)

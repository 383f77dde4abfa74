"""Compile the C oracle into oracle/liborc.so with gcc.

The oracle is test infrastructure: the product library never links it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "crop_oracle.c")
LIB = os.path.join(HERE, "liborc.so")


CPU_SRC = os.path.join(HERE, "crop_cpu.c")
CPU_LIB = os.path.join(HERE, "libcropcpu.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    build_cpu(verbose)
    return LIB


def build_cpu(verbose: bool = False) -> str:
    """The paper's method on the host (the benchmark's multi-core CPU
    baseline).  -march=x86-64-v3 (AVX2) rather than native: the library is
    built in one container and timed on another host."""
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=c11", "-fPIC", "-shared", "-pthread",
           "-Wall", "-Wextra", "-o", CPU_LIB + ".tmp", CPU_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CPU_LIB + ".tmp", CPU_LIB)
    return CPU_LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

"""Build step for the CPU oracle (test infrastructure): compiles lbm_oracle.c
into oracle/liblbm_oracle.so with gcc, FP64, no fast-math, no FMA contraction."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")
CFLAGS = ["-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wextra", "-D_GNU_SOURCE"]


def compile_source(src: str, lib: str, verbose: bool = False) -> str:
    """Compile one C source of the oracle into the shared library `lib`."""
    cmd = ["gcc", *CFLAGS, "-I", HERE, src, "-o", lib + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def build(verbose: bool = False) -> str:
    return compile_source(SRC, LIB, verbose)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

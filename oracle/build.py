"""Compile the C oracle into oracle/liboracle.so with gcc (FP64, no contraction)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tlmpm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def compile_source(src, out):
    """gcc the oracle source file `src` into the shared library `out` (OpenMP on the
    loops with independent iterations; orc_set_threads picks the thread count)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-Wall", "-Wno-unused-function", "-o", out + ".tmp", src, "-lm"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def build(force=True):
    """Build liboracle.so; with force=False only when missing or stale."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    return compile_source(SRC, LIB)


if __name__ == "__main__":
    print(build())

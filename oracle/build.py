"""Compile the C oracle (D2Q9 and D3Q19) into ``oracle/_build/liborc.so`` with gcc.

TEST INFRASTRUCTURE (see the package docstring).  Flags: -O2, no FMA
contraction, no fast math, OpenMP for the row loop of the step (used only when
timing the oracle; results do not depend on the thread count).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
SRC3 = os.path.join(HERE, "lbm3d_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liborc.so")

CFLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile (always when ``force``) and return the library path."""
    if (not force and os.path.exists(LIB) and
            os.path.getmtime(LIB) >= max(os.path.getmtime(SRC), os.path.getmtime(SRC3))):
        return LIB
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, SRC, SRC3, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Only gcc and libm/OpenMP are used; nothing here touches the HIP library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rvea_oracle.c")
SRCS = [SRC, os.path.join(HERE, "indicators.c"), os.path.join(HERE, "operators.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
        [os.path.getmtime(f) for f in SRCS] + [os.path.getmtime(os.path.join(HERE, "rvea_oracle.h"))]
    ):
        return LIB
    cmd = [
        "gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fopenmp",
        "-fPIC", "-shared", "-Wall", "-o", LIB + ".tmp", *SRCS, "-lm",
    ]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv))

"""Compile the C oracle into ``oracle/libgift_oracle.so`` (test infrastructure).

Plain gcc, ``-O2 -ffp-contract=off``: no fused multiply-adds, so every FP64
operation rounds exactly as written in the C source.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gift_oracle.c")
LIB = os.path.join(HERE, "libgift_oracle.so")


def build(out: str = LIB, src: str = SRC, extra=()) -> str:
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", tmp, src, "-lm", *extra]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(*sys.argv[1:2]))

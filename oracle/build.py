"""Compile the CPU oracle (plain C) into oracle/liboracle.so with gcc."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bcf_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")
CMD = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", OUT, SRC]


def build(out: str = OUT, src: str = SRC, extra=()) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra", *extra, "-o", out, src]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(), file=sys.stderr)

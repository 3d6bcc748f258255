"""Build the CPU oracle shared library (test infrastructure).

Compiles ``plds_oracle.c`` with gcc into ``libplds_oracle.so`` next to this file.
The oracle is plain single-threaded C; -O2 as for the CPU baseline.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "plds_oracle.c")
LIB = os.path.join(HERE, "libplds_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-g", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

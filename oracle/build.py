"""Compile the oracle's C sources (plain gcc, no GPU code)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SV_SRC = os.path.join(HERE, "sv.c")
SV_LIB = os.path.join(HERE, "_sv.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(SV_LIB) and os.path.getmtime(SV_LIB) >= os.path.getmtime(SV_SRC):
        return SV_LIB
    tmp = SV_LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", SV_SRC, "-o", tmp],
                   check=True)
    os.replace(tmp, SV_LIB)
    return SV_LIB


if __name__ == "__main__":
    print(build())

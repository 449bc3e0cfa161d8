"""Compile the CPU oracle library (test infrastructure)."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build_oracle(force: bool = True) -> str:
    src = os.path.join(_HERE, "spgemm_oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, src]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_oracle(force=True))

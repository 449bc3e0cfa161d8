"""Compile the CPU oracle library (test infrastructure)."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


# AddressSanitizer + UndefinedBehaviorSanitizer build (host code only, for the
# sanitized run of the pin tests): any finding aborts the process.
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all"]


def build_oracle(force: bool = True, sanitize: bool = False, out: str = "") -> str:
    src = os.path.join(_HERE, "spgemm_oracle.c")
    out = out or os.path.join(_HERE, "liboracle_san.so" if sanitize else "liboracle.so")
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        opt = SANITIZE_FLAGS if sanitize else ["-O2"]
        cmd = ["gcc", *opt, "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, src]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_oracle(force=True))

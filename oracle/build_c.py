"""Compile the oracle's C part (sinkhorn.c) into oracle/liboracle_sinkhorn.so
with gcc (-O2, OpenMP; -fno-math-errno lets the exponential loop use the
C library's vector exp).  Test infrastructure: only the oracle loads it."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sinkhorn.c")
OUT = os.path.join(HERE, "liboracle_sinkhorn.so")


def build() -> str:
    tmp = OUT + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fno-math-errno", "-fPIC", "-shared", "-o", tmp, SRC, "-lm", "-lmvec"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"oracle C build failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())

"""Algorithmic FP64 flop counts of the sweep kernels' own arithmetic.

Compiles flopcount.cpp (host only) against the kernels' templated math
headers with an operation-counting real type, runs it, and returns the
counts per cell-update.  These counts are the per-unit figures behind the
roofline numbers of bench.py."""
from __future__ import annotations

import functools
import json
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "..", "_build", "flopcount")


@functools.lru_cache(maxsize=1)
def counts() -> dict:
    src = os.path.join(HERE, "flopcount.cpp")
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    if not os.path.exists(EXE) or os.path.getmtime(EXE) < max(
            os.path.getmtime(os.path.join(HERE, "..", "csrc", f))
            for f in os.listdir(os.path.join(HERE, "..", "csrc"))) or \
            os.path.getmtime(EXE) < os.path.getmtime(src):
        subprocess.run(["hipcc", "-x", "hip", "--offload-host-only", "-O1", "-std=c++17",
                        "-o", EXE, src], check=True)
    out = subprocess.run([EXE], check=True, capture_output=True, text=True).stdout
    return {d["path"]: d for d in map(json.loads, out.strip().splitlines())}


def euler1d_cell_update(full: bool = True) -> dict:
    return counts()["euler1d_nonlinear_charwise" if full else "euler1d_linear"]


def euler2d_cell_update(full: bool = True) -> dict:
    return counts()["euler2d_nonlinear_charwise" if full else "euler2d_linear"]


if __name__ == "__main__":
    for k, v in counts().items():
        print(k, v)

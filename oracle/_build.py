"""Build step for the oracle's C source (gcc, FP64, OpenMP, no fast-math).

Test infrastructure: compiled by the package build step so the checker is
ready, and called only by tests, the smoke check and the CPU baseline.
"""
from __future__ import annotations

import pathlib
import subprocess

HERE = pathlib.Path(__file__).resolve().parent
SRC = HERE / "rtm_oracle.c"
OUT = HERE / "liboracle.so"

CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = False) -> pathlib.Path:
    if force or not OUT.exists() or OUT.stat().st_mtime < SRC.stat().st_mtime:
        tmp = OUT.with_suffix(".so.tmp")
        subprocess.run(["gcc", *CFLAGS, str(SRC), "-o", str(tmp), "-lm"], check=True)
        tmp.replace(OUT)
    return OUT


if __name__ == "__main__":
    print(build(force=True))

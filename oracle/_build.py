"""Build step for the oracle's C sources (gcc, no fast-math, no contraction).

Test infrastructure: compiled by the package build step so the checker is
ready, and called only by tests, the smoke check and the CPU baseline.
"""
from __future__ import annotations

import pathlib
import subprocess

HERE = pathlib.Path(__file__).resolve().parent
SRCS = [HERE / "rtm_oracle.c", HERE / "bet_oracle.c"]
OUT = HERE / "liboracle.so"

CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = False) -> pathlib.Path:
    newest = max(s.stat().st_mtime for s in SRCS)
    if force or not OUT.exists() or OUT.stat().st_mtime < newest:
        tmp = OUT.with_suffix(".so.tmp")
        subprocess.run(["gcc", *CFLAGS, *map(str, SRCS), "-o", str(tmp), "-lm"], check=True)
        tmp.replace(OUT)
    return OUT


if __name__ == "__main__":
    print(build(force=True))

"""Build step of the HIP library: hipcc for gfx950 -> paper_2001_06444_amd/librtm.so."""
from __future__ import annotations

import os
import pathlib
import subprocess

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
OUT = PKG / "librtm.so"
SOURCES = [CSRC / "rtm_kernels.hip", CSRC / "rtm_aux.hip", CSRC / "rtm_codec.hip", CSRC / "rtm_zfp.hip",
           CSRC / "rtm_bet.hip", CSRC / "rtm_runtime.hip"]
HEADERS = [CSRC / "rtm_internal.h", CSRC / "rtm_codec.h", CSRC / "rtm_zfp.h", CSRC / "rtm_bet.h", CSRC / "rtm_device.h", CSRC / "rtm_arena.h", CSRC / "rtm_sched.h", ROOT / "include" / "rtm.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (their forms have produced silent wrong results)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-I", str(ROOT / "include"),
]


def build(force: bool = True, verbose: bool = False) -> pathlib.Path:
    newest = max(p.stat().st_mtime for p in SOURCES + HEADERS)
    if not force and OUT.exists() and OUT.stat().st_mtime >= newest:
        return OUT
    tmp = OUT.with_name(OUT.name + ".tmp")
    # roctx: named ranges of the scheduler and the batched phases for profiler timelines
    cmd = [HIPCC, *FLAGS, *map(str, SOURCES), "-o", str(tmp), "-lpthread", "-L/opt/rocm/lib",
           "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    tmp.replace(OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))

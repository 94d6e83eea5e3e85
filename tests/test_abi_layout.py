"""The Python binding's ctypes structures match the C ABI's structs in
include/rtm.h field for field: a C program built with the host compiler
from the header prints every field's offset and every struct's size, and
the binding's layouts must equal them (a field added on one side only, or
a type changed, shifts an offset or a size and fails here).  CPU only."""
import ctypes
import pathlib
import subprocess

import pytest

from paper_2001_06444_amd import rtm

ROOT = pathlib.Path(__file__).resolve().parents[1]

PAIRS = {"Grid": "rtm_grid", "Point": "rtm_point", "ImgOpts": "rtm_img_opts", "ShotDesc": "rtm_shot_desc",
         "BornShot": "rtm_born_shot", "Job": "rtm_job", "JobInfo": "rtm_job_info", "CtxStats": "rtm_ctx_stats_t",
         "BetConfig": "rtm_bet_config", "BetChainInfo": "rtm_bet_chain_info"}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "rtm.h"', "int main(void) {"]
    for py, c in PAIRS.items():
        lines.append(f'  printf("{py} sizeof %zu\\n", sizeof({c}));')
        for f in getattr(rtm, py)._fields_:
            lines.append(f'  printf("{py} {f[0]} %zu\\n", offsetof({c}, {f[0]}));')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c11", "-I", str(ROOT / "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {(a, b): int(v) for a, b, v in (ln.split() for ln in out.splitlines())}


@pytest.mark.parametrize("py", sorted(PAIRS))
def test_binding_struct_matches_header(c_layout, py):
    cls = getattr(rtm, py)
    assert ctypes.sizeof(cls) == c_layout[(py, "sizeof")], (py, ctypes.sizeof(cls), c_layout[(py, "sizeof")])
    for f in cls._fields_:
        assert getattr(cls, f[0]).offset == c_layout[(py, f[0])], (py, f[0])

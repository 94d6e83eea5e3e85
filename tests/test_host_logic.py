"""Host logic of the runtime built with g++ and the sanitizers (CPU only):
the arena allocator under a long random alloc/release sequence (ASan +
UBSan) and under eight concurrent threads (TSan)."""
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
SRC = ROOT / "tests" / "host" / "arena_stress.cpp"
INC = ROOT / "paper_2001_06444_amd" / "csrc"


def _build_and_run(tmp_path, flags, args):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "arena_stress"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, f"-I{INC}",
           str(SRC), "-o", str(exe), "-pthread"]
    subprocess.run(cmd, check=True)
    r = subprocess.run([str(exe), *args], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_arena_single_threaded_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"], [])
    assert "single:" in out


def test_arena_concurrent_tsan(tmp_path):
    out = _build_and_run(tmp_path, ["-fsanitize=thread"], ["threaded"])
    assert "threaded:" in out

"""Host logic built with the sanitizers (CPU only):
  - the arena allocator under a long random alloc/release sequence (ASan +
    UBSan) and under eight concurrent threads (TSan);
  - the serving engine's job bookkeeping (rtm_sched.h) against its rules
    with a mock clock (ASan + UBSan) and under concurrent submitters,
    pollers, a canceller and a scheduler thread (TSan, and ASan);
  - the oracle's C code (oracle/rtm_oracle.c, oracle/bet_oracle.c) through
    every entry point on small and degenerate grids (ASan + UBSan)."""
import os
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
HOST = ROOT / "tests" / "host"
SRC = HOST / "arena_stress.cpp"
INC = ROOT / "paper_2001_06444_amd" / "csrc"
ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _build_and_run(tmp_path, flags, args, src=SRC):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / src.stem
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, f"-I{INC}",
           str(src), "-o", str(exe), "-pthread"]
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


def test_job_book_rules_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, ASAN, [], HOST / "sched_test.cpp")
    assert "rules: ok" in out


def test_job_book_concurrent_tsan(tmp_path):
    out = _build_and_run(tmp_path, ["-fsanitize=thread"], ["threaded"], HOST / "sched_test.cpp")
    assert "threaded:" in out


def test_job_book_concurrent_asan(tmp_path):
    out = _build_and_run(tmp_path, ASAN, ["threaded"], HOST / "sched_test.cpp")
    assert "threaded:" in out


@pytest.mark.parametrize("driver", ["oracle_rtm_asan.c", "oracle_bet_asan.c"])
def test_oracle_c_asan_ubsan(tmp_path, driver):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path / driver[:-2]
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off", *ASAN, str(HOST / driver),
                    "-o", str(exe), "-lm"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env={**os.environ, "OMP_NUM_THREADS": "2"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert ": ok" in r.stdout

"""bench.py behaviour that needs no GPU: the one-GPU rule and the check that
keeps a committed traffic record from being reported for other sources."""
import json
import pathlib
import subprocess
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_traffic_record_is_dropped_when_its_sources_change(tmp_path, monkeypatch):
    import bench

    src = tmp_path / "kernel.hip"
    src.write_text("// version 1\n")
    monkeypatch.setattr(bench, "ROOT", tmp_path)
    (tmp_path / "profiles").mkdir()
    rec = {"kernel_source_hash": bench.kernel_source_hash(("kernel.hip",)), "hbm_bytes_per_launch": 123.0}
    (tmp_path / "profiles" / "t.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("t.json", ("kernel.hip",)) == pytest.approx(123.0)
    src.write_text("// version 2\n")
    assert bench.measured_traffic("t.json", ("kernel.hip",)) is None
    assert bench.measured_traffic("missing.json", ("kernel.hip",)) is None

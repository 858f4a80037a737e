"""CPU checks of bench.py's contract that need no GPU: more than one GPU is
refused with a message, the recorded HBM traffic is only reported while the
profiled kernel sources are unchanged, and the percentile helper is the
nearest-rank one."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_recorded_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    # The committed summary matches the committed sources.
    assert isinstance(bench.recorded_traffic(), int)
    # A summary taken from other sources is not used.
    text = open(bench.TRAFFIC_FILE).read()
    stale = tmp_path / "stale.md"
    stale.write_text(text.replace(bench.kernel_source_hash(), "0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.recorded_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.recorded_traffic() is None


def test_percentile_is_nearest_rank():
    xs = [5.0, 1.0, 4.0, 2.0, 3.0]
    assert bench.pct(xs, 50) == 3.0
    assert bench.pct(xs, 100) == 5.0
    assert bench.pct(xs, 1) == 1.0
    assert bench.pct(list(range(1, 101)), 99) == 99
    assert bench.pct([1.0, 2.0, 3.0, 4.0], 50) == 2.0

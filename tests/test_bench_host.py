"""Host-side logic of bench.py (CPU only): the one-GPU guard, and the
recorded HBM traffic, reported only while the match kernel's sources hash as
they did when the counters were taken."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_recorded_traffic_follows_the_source_hash(monkeypatch):
    assert bench.recorded_traffic("no_such_workload", "learned") is None
    assert bench.recorded_traffic("plain_1m", "given") is None   # the counters were taken on another plan
    got = bench.recorded_traffic("plain_1m", "learned")
    if got is not None:   # the committed summary matches the committed sources
        assert got > 0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.recorded_traffic("plain_1m", "learned") is None

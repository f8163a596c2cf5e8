"""Host-side logic of bench.py (CPU only): the one-GPU guard, the recorded
HBM traffic, reported only while the match kernel's sources hash as they did
when the counters were taken, and the test that keeps rule sets which tell t
from s out of the per-pair network's leg."""
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


def test_ordered_rules_detects_rules_that_tell_t_from_s():
    """The per-pair network's leg runs only on rule sets of predicates that
    compare one attribute of both tuples."""
    from gen import CONTAIN, ED_CROSS, EQ, EQ_CONST, EQ_CROSS, JACCARD_CROSS, Pred
    from gen.workloads import plain_1m_ordered_rules
    assert not bench.ordered_rules([[Pred(EQ, 0), Pred(EQ_CROSS, 1, attr_b=1)], [Pred(ED_CROSS, 2, k=1, attr_b=2)]])
    assert not bench.ordered_rules([[Pred(JACCARD_CROSS, 2, q=2, num=1, den=2, attr_b=2)]])
    for p in (Pred(EQ_CONST, 1, c=3), Pred(EQ_CROSS, 1, attr_b=0), Pred(ED_CROSS, 0, k=1, attr_b=2),
              Pred(JACCARD_CROSS, 0, q=2, num=1, den=2, attr_b=2), Pred(CONTAIN, 0, q=2, num=1, den=2, attr_b=0)):
        assert bench.ordered_rules([[Pred(EQ, 3), p]]), p
    assert bench.ordered_rules(plain_1m_ordered_rules())

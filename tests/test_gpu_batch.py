"""GPU tests of batched matching: many relations and rule sets in one
persistent work-stealing launch (graph-captured, autotuned) give, per job,
exactly the oracle's pair set; graph replays interleaved with other work
stay exact; the output-capacity regrow path; stale handles."""
import numpy as np
import pytest

import oracle
from gen import EQ, Pred, workloads
from learned_util import train_model

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_04349_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(hb):
    c = hb.hb_create(0, allocator="torch")
    yield c
    c.close()


def load_jobs(hb, ctx, jobs):
    ids = []
    for rel, rules in jobs:
        rid = hb.hb_load_relation(ctx, rel.columns, rel.n_rows)
        rs = hb.hb_compile_rules(ctx, rid, rules)
        hb.hb_partition(ctx, rid, rs)
        ids.append((rid, rs))
    return ids


@pytest.fixture(scope="module")
def batched(hb, ctx):
    jobs = workloads.batched_64(scale=0.005, cap=100)
    want = [oracle.blocking(rel, rules, threads=16) for rel, rules in jobs]
    ids = load_jobs(hb, ctx, jobs)
    return jobs, want, ids


def test_batch_matches_oracle(hb, ctx, batched):
    jobs, want, ids = batched
    print(f"[gpu-case] batch of {len(jobs)} jobs, graph + autotune", flush=True)
    bid = hb.hb_batch_create(ctx, ids, "heuristic", graph=True, autotune=True)
    info = hb.hb_batch_info(ctx, bid)
    print(f"[gpu-case] {info}", flush=True)
    assert info["graph"] and info["n_jobs"] == len(jobs) and len(info["tune_ms"]) > 0
    total = hb.hb_batch_run(ctx, bid)
    assert total == sum(len(w) for w in want)
    for k in range(len(jobs)):
        assert np.array_equal(hb.hb_batch_result(ctx, bid, k), want[k]), k
    hb.hb_batch_destroy(ctx, bid)


def test_batch_graph_replays_with_work_between(hb, ctx, batched):
    jobs, want, ids = batched
    print("[gpu-case] graph replays", flush=True)
    bid = hb.hb_batch_create(ctx, ids, "heuristic", graph=True)
    for rep in range(3):
        hb.hb_batch_run(ctx, bid)
        for k in range(0, len(jobs), 7):
            assert np.array_equal(hb.hb_batch_result(ctx, bid, k), want[k]), (rep, k)
        # eager work on the same context between replays
        rid, rs = ids[rep]
        assert np.array_equal(hb.hb_match(ctx, rid, rs, "given"), want[rep])
    hb.hb_batch_destroy(ctx, bid)


def test_batch_without_graph_and_learned(hb, ctx, batched):
    jobs, want, ids = batched
    print("[gpu-case] learned plan batch, no graph", flush=True)
    assert np.isfinite(train_model(hb, ctx))
    bid = hb.hb_batch_create(ctx, ids[:24], "learned", graph=False)
    hb.hb_batch_run(ctx, bid)
    for k in range(24):
        assert np.array_equal(hb.hb_batch_result(ctx, bid, k), want[k]), k
    hb.hb_batch_destroy(ctx, bid)


def test_batch_multi_key_and_regrow(hb, ctx):
    print("[gpu-case] multi-key jobs and output regrow", flush=True)
    jobs = [workloads.random_small(3000 + s, n=300, n_keys=1 + s % 3) for s in range(6)]
    # every candidate pair matches: far more pairs than the first capacity
    rel, _ = workloads.plain_1m(n=3000)
    jobs.append((rel, [[Pred(EQ, 3)]]))
    want = [oracle.blocking(r, ru, threads=16) for r, ru in jobs]
    assert len(want[-1]) > 65536
    ids = load_jobs(hb, ctx, jobs)
    bid = hb.hb_batch_create(ctx, ids, "heuristic", graph=True)
    for _ in range(2):
        hb.hb_batch_run(ctx, bid)
        for k in range(len(jobs)):
            assert np.array_equal(hb.hb_batch_result(ctx, bid, k), want[k]), k
    hb.hb_batch_destroy(ctx, bid)
    for rid, _ in ids:
        hb.hb_release_relation(ctx, rid)


def test_batch_stale_relation(hb, ctx):
    rel, rules = workloads.person_small()
    ids = load_jobs(hb, ctx, [(rel, rules)])
    bid = hb.hb_batch_create(ctx, ids, "heuristic", graph=False)
    hb.hb_release_relation(ctx, ids[0][0])
    with pytest.raises(hb.HbError) as e:
        hb.hb_batch_run(ctx, bid)
    assert e.value.status == hb.HB_ERR_STALE_ID
    hb.hb_batch_destroy(ctx, bid)
    with pytest.raises(hb.HbError):
        hb.hb_batch_destroy(ctx, bid)

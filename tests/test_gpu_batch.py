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
    hb.hb_set_learned_min_saving(c, 0.0)   # every per-block plan kept: their parity
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


@pytest.mark.parametrize("form,graph", [("streams", True), ("multi", False), ("persistent", True)])
def test_batch_each_form_matches_oracle(hb, ctx, batched, form, graph):
    """Every launch form, forced, on a mix of the batched jobs, a two-key
    job and a long-title job (edit-distance patterns past 64 bytes, the
    Myers state in LDS for the queue kernels, in registers for the
    per-partition launches)."""
    jobs, want, ids = batched
    print(f"[gpu-case] forced form {form}, graph {graph}", flush=True)
    extra = [workloads.random_small(4100, n=400, n_keys=2), workloads.long_titles_5m(n=3000)]
    extra_want = [oracle.blocking(r, ru, threads=16) for r, ru in extra]
    extra_ids = load_jobs(hb, ctx, extra)
    sel = list(range(0, len(jobs), 4))
    bid = hb.hb_batch_create(ctx, [ids[k] for k in sel] + extra_ids, "heuristic", graph=graph, form=form)
    info = hb.hb_batch_info(ctx, bid)
    assert info["form"] == form
    hb.hb_batch_run(ctx, bid)
    for x, k in enumerate(sel):
        assert np.array_equal(hb.hb_batch_result(ctx, bid, x), want[k]), (form, k)
    for x in range(len(extra)):
        assert np.array_equal(hb.hb_batch_result(ctx, bid, len(sel) + x), extra_want[x]), (form, "extra", x)
    hb.hb_batch_destroy(ctx, bid)
    for rid, _ in extra_ids:
        hb.hb_release_relation(ctx, rid)


def test_batch_forced_form_with_autotune_rejected(hb, ctx, batched):
    _, _, ids = batched
    with pytest.raises(hb.HbError) as e:
        hb.hb_batch_create(ctx, ids[:2], "heuristic", graph=False, autotune=True, form="multi")
    assert e.value.status == hb.HB_ERR_INVALID_ARG


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


class _Col:
    pass


def pinned_columns(rel, torch):
    """The relation's arrays copied into pinned host memory."""
    out = []
    for c in rel.columns:
        d = _Col()
        d.type = c.type
        for name in ("offsets", "data", "values", "valid"):
            a = getattr(c, name)
            if name == "offsets" and a is not None:
                a = a.view(np.int64)
            setattr(d, name, torch.from_numpy(np.ascontiguousarray(a)).pin_memory() if a is not None and len(a)
                    else None)
        out.append(d)
    return out


def test_async_load_matches_oracle(hb, ctx):
    import torch
    print("[gpu-case] asynchronous loads", flush=True)
    cases = [workloads.person_small()] + [workloads.random_small(4000 + s, n=250, n_keys=1 + s % 3)
                                          for s in range(4)]
    held, ids = [], []
    for k, (rel, rules) in enumerate(cases):
        cols = pinned_columns(rel, torch) if k % 2 == 0 else rel.columns
        held.append(cols)
        ids.append(hb.hb_load_relation_async(ctx, cols, rel.n_rows))
    for (rel, rules), rid in zip(cases, ids):
        rs = hb.hb_compile_rules(ctx, rid, rules)
        hb.hb_partition(ctx, rid, rs)
        assert np.array_equal(hb.hb_match(ctx, rid, rs, "heuristic"), oracle.blocking(rel, rules, threads=16))
        hb.hb_release_relation(ctx, rid)


def test_async_load_invalid_offsets_reported_on_use(hb, ctx):
    rel, rules = workloads.person_small()
    col = rel.columns[0]
    bad = col.offsets.copy()
    bad[10], bad[11] = bad[11], bad[10]   # decreasing once; the last offset is unchanged
    cols = list(rel.columns)
    c0 = _Col()
    c0.type, c0.offsets, c0.data, c0.values, c0.valid = col.type, bad, col.data, None, None
    cols[0] = c0
    rid = hb.hb_load_relation_async(ctx, cols, rel.n_rows)
    with pytest.raises(hb.HbError) as e:
        hb.hb_compile_rules(ctx, rid, rules)
    assert e.value.status == hb.HB_ERR_INVALID_ARG
    hb.hb_release_relation(ctx, rid)


def test_async_pipeline_chunks(hb, ctx):
    """A relation split by key into chunks (no block spans two), each loaded
    asynchronously while the previous one is matched: the union of the
    chunks' results, mapped back to global rows, equals the oracle's."""
    import torch
    print("[gpu-case] chunked pipeline", flush=True)
    rel, rules = workloads.long_titles_5m(n=30_000)
    want = oracle.blocking(rel, rules, threads=16)
    key = rel.columns[0].values
    chunks = [np.flatnonzero(key % 4 == m) for m in range(4)]
    parts = [rel.take(rows) for rows in chunks]
    pinned = [pinned_columns(p, torch) for p in parts]
    got = []
    nxt = hb.hb_load_relation_async(ctx, pinned[0], parts[0].n_rows)
    for k in range(len(parts)):
        cur = nxt
        if k + 1 < len(parts):
            nxt = hb.hb_load_relation_async(ctx, pinned[k + 1], parts[k + 1].n_rows)
        rs = hb.hb_compile_rules(ctx, cur, rules)
        hb.hb_partition(ctx, cur, rs)
        local = hb.hb_match(ctx, cur, rs, "heuristic")
        i = chunks[k][(local >> np.uint64(32)).astype(np.int64)]
        j = chunks[k][(local & np.uint64(0xFFFFFFFF)).astype(np.int64)]
        got.append((np.minimum(i, j).astype(np.uint64) << np.uint64(32)) | np.maximum(i, j).astype(np.uint64))
        hb.hb_release_relation(ctx, cur)
    assert np.array_equal(np.sort(np.concatenate(got)), want)

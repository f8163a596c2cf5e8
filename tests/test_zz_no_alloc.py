"""hb_match_noalloc (the allocation-free variant of hb_match) against
hb_match itself, through the C ABI: equal sorted pair lists on two calls in
a row, the second on a smaller relation, with no device allocation asked of
the context's allocator during either call; the refused plan and the
capacity protocol."""
import numpy as np
import pytest

from gen import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_04349_amd as m
    return m


def prepared(hb, ctx, rel, rules):
    rid = hb.hb_load_relation(ctx, rel.columns, rel.n_rows)
    rs = hb.hb_compile_rules(ctx, rid, rules)
    hb.hb_partition(ctx, rid, rs)
    return rid, rs


def noalloc(hb, ctx, rid, rs, plan, out):
    import torch
    torch.cuda.synchronize()
    before = ctx.alloc_calls
    n = hb.hb_match_noalloc(ctx, rid, rs, plan, out)
    assert ctx.alloc_calls == before, "hb_match_noalloc asked the allocator for device memory"
    return out[:n].cpu().numpy().view(np.uint64).copy()


def test_noalloc_equals_match_two_calls(hb):
    import torch
    ctx = hb.hb_create(0, allocator="torch")
    try:
        out = torch.full((1 << 20,), -1, dtype=torch.int64, device="cuda")
        # first call: a 60k draw of the plain recipe (blocks of several 64 x 64
        # tiles with ragged tails, five rules)
        rel, rules = workloads.plain_1m(n=60_000)
        rid, rs = prepared(hb, ctx, rel, rules)
        print(f"[gpu-case] noalloc call 1: {rel.n_rows} tuples, heuristic plan", flush=True)
        got1 = noalloc(hb, ctx, rid, rs, "heuristic", out)
        want1 = hb.hb_match(ctx, rid, rs, "heuristic")
        assert len(want1) > 100
        assert np.array_equal(got1, want1)
        # second call: a smaller relation (the array keeps the first call's
        # contents), another plan
        rel2, rules2 = workloads.person_small()
        rid2, rs2 = prepared(hb, ctx, rel2, rules2)
        print(f"[gpu-case] noalloc call 2: {rel2.n_rows} tuples, given plan", flush=True)
        got2 = noalloc(hb, ctx, rid2, rs2, "given", out)
        want2 = hb.hb_match(ctx, rid2, rs2, "given")
        assert 0 < len(want2) < len(want1)
        assert np.array_equal(got2, want2)
        # and the first relation again, after the smaller one
        assert np.array_equal(noalloc(hb, ctx, rid, rs, "selective", out), want1)
    finally:
        ctx.close()


def test_noalloc_ordered_two_keys_and_errors(hb):
    import torch
    ctx = hb.hb_create(0, allocator="torch")
    try:
        out = torch.empty(1 << 20, dtype=torch.int64, device="cuda")
        rel, _ = workloads.plain_1m(n=40_000)
        rid, rs = prepared(hb, ctx, rel, workloads.plain_1m_ordered_rules())
        print("[gpu-case] noalloc ordered rule set, 40k tuples", flush=True)
        assert np.array_equal(noalloc(hb, ctx, rid, rs, "heuristic", out), hb.hb_match(ctx, rid, rs, "heuristic"))
        rel2, rules2 = workloads.learned_10m(n=60_000)
        rid2, rs2 = prepared(hb, ctx, rel2, rules2)
        print("[gpu-case] noalloc two keys, 60k tuples", flush=True)
        want = hb.hb_match(ctx, rid2, rs2, "heuristic")
        assert np.array_equal(noalloc(hb, ctx, rid2, rs2, "heuristic", out), want)
        with pytest.raises(hb.HbError) as e:
            hb.hb_match_noalloc(ctx, rid2, rs2, "learned", out)
        assert e.value.status == hb.HB_ERR_INVALID_ARG
        with pytest.raises(hb.HbError) as e:
            hb.hb_match_noalloc(ctx, rid2, rs2, "heuristic", out, capacity=len(want) - 1)
        assert e.value.status == hb.HB_ERR_CAPACITY
    finally:
        ctx.close()

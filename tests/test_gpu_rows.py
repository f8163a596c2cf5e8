"""GPU parity of the launch shapes of hb_set_rows_per_wave (with small
blocks packed into shared tiles, hb_set_pack_small_blocks) (16 i-rows per
wave batch, four batches per 64 x 64 tile; 32, two batches; 64, one batch
with 64-bit row masks, the default, which the rest of the suite runs): bit-exact against the oracle on block
sizes around the batch and tile edges, random small relations, patterns
past 64 bytes, several tiles per block, two keys, the learned plan and the
allocation-free entry point; the option is refused for other values."""
import numpy as np
import pytest

import oracle
from gen import ABSDIFF, CATEGORICAL, ED, EQ, JACCARD, Pred, Relation, int_column, string_column
from gen import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_04349_amd as m
    return m


@pytest.fixture(scope="module", params=[16, 32, 64])
def ctx(hb, request):
    c = hb.hb_create(0, allocator="torch")
    hb.hb_set_rows_per_wave(c, request.param)
    hb.hb_set_learned_min_saving(c, 0.0)   # every per-block plan kept: their parity
    hb.hb_set_pack_small_blocks(c, True)   # small blocks packed into shared tiles: their parity
    c.rows = request.param
    yield c
    c.close()


def run(hb, ctx, rel, rules, plan):
    rid = hb.hb_load_relation(ctx, rel.columns, rel.n_rows)
    rs = hb.hb_compile_rules(ctx, rid, rules)
    n_cand = hb.hb_partition(ctx, rid, rs)
    out = hb.hb_match(ctx, rid, rs, plan)
    hb.hb_release_relation(ctx, rid)
    return out, n_cand


def show(ctx, case):
    print(f"[gpu-case] rows={ctx.rows} {case}", flush=True)


def test_block_size_sweep_rows(hb, ctx):
    show(ctx, "block size sweep")
    r = np.random.default_rng(17)
    sizes = [1, 2, 3, 15, 16, 17, 31, 32, 33, 47, 48, 49, 63, 64, 65, 95, 96, 97, 127, 128, 129, 200]
    keys = np.concatenate([np.full(n, 1000 + k) for k, n in enumerate(sizes)])
    r.shuffle(keys)
    n = len(keys)
    strings = [bytes(r.integers(97, 100, size=int(r.integers(4, 12))).astype(np.uint8)) for _ in range(n)]
    ints = [int(v) for v in r.integers(0, 20, size=n)]
    rel = Relation([string_column("s", strings), int_column("k", keys.tolist(), CATEGORICAL),
                    int_column("i", ints)], n)
    for rules in ([[Pred(EQ, 1)]],
                  [[Pred(EQ, 1), Pred(ED, 0, k=2)], [Pred(EQ, 1), Pred(ABSDIFF, 2, d=1)]],
                  [[Pred(EQ, 1), Pred(JACCARD, 0, q=2, num=1, den=2), Pred(ABSDIFF, 2, d=5)]],
                  [[Pred(EQ, 1), Pred(ABSDIFF, 2, d=3), Pred(ED, 0, k=3)],
                   [Pred(EQ, 1), Pred(ABSDIFF, 2, d=3), Pred(JACCARD, 0, q=2, num=2, den=5)]]):
        want = oracle.blocking(rel, rules)
        for plan in ("given", "heuristic"):
            got, n_cand = run(hb, ctx, rel, rules, plan)
            assert n_cand == sum(m * (m - 1) // 2 for m in sizes)
            assert np.array_equal(got, want), (rules, plan)


@pytest.mark.parametrize("seed", range(10))
def test_random_small_rows(hb, ctx, seed):
    kw = dict(n=400 if seed % 3 else 150, long_strings=seed % 4 != 3, n_keys=1 + seed % 3,
              alphabet=b"ab" if seed % 2 else b"abc", n_key_values=4 if seed % 5 == 0 else 8,
              n_rules=2 + seed % 5, null_p=0.0 if seed % 7 == 0 else 0.05)
    show(ctx, f"random_small seed={seed}")
    rel, rules = workloads.random_small(3000 + seed, **kw)
    want = oracle.blocking(rel, rules, threads=8)
    for plan in ("given", "heuristic", "selective"):
        got, _ = run(hb, ctx, rel, rules, plan)
        assert np.array_equal(got, want), plan


def test_long_patterns_rows(hb, ctx):
    """Edit-distance patterns past 64 bytes (the register-state kernel)."""
    show(ctx, "long patterns")
    rel, rules = workloads.long_titles_5m(n=30_000)
    want = oracle.blocking(rel, rules, threads=8)
    got, _ = run(hb, ctx, rel, rules, "heuristic")
    assert np.array_equal(got, want)


def test_two_keys_learned_and_noalloc_rows(hb, ctx):
    """The two-key recipe with guard groups, the learned plan (its choice
    priced at 32 rows) and hb_match_noalloc."""
    import torch

    from learned_util import train_model
    show(ctx, "two keys, learned, noalloc")
    rel, rules = workloads.learned_10m(n=40_000)
    want = oracle.blocking(rel, rules, threads=16)
    assert np.isfinite(train_model(hb, ctx))
    rid = hb.hb_load_relation(ctx, rel.columns, rel.n_rows)
    rs = hb.hb_compile_rules(ctx, rid, rules)
    hb.hb_partition(ctx, rid, rs)
    for plan in ("heuristic", "learned"):
        assert np.array_equal(hb.hb_match(ctx, rid, rs, plan), want), plan
    out = torch.empty(1 << 20, dtype=torch.int64, device="cuda")
    n = hb.hb_match_noalloc(ctx, rid, rs, "heuristic", out)
    assert np.array_equal(out[:n].cpu().numpy().view(np.uint64), want)
    hb.hb_release_relation(ctx, rid)


def test_plain_several_tiles_rows(hb, ctx):
    show(ctx, "plain 40k")
    rel, rules = workloads.plain_1m(n=40_000)
    want = oracle.blocking(rel, rules, threads=8)
    got, _ = run(hb, ctx, rel, rules, "heuristic")
    assert np.array_equal(got, want)


def test_rows_option_refused(hb, ctx):
    for bad in (0, 8, 128):
        with pytest.raises(hb.HbError) as e:
            hb.hb_set_rows_per_wave(ctx, bad)
        assert e.value.status == hb.HB_ERR_INVALID_ARG


_ORACLE = {}   # oracle results shared by the parametrized cases


def test_launch_settings_refused(hb, ctx):
    """The per-lane threshold above 32 and a minimum saving outside [0, 1)
    are refused; accepted values leave the result unchanged (covered by the
    sweeps above at the defaults)."""
    with pytest.raises(hb.HbError) as e:
        hb.hb_set_sparse_rows(ctx, 33)
    assert e.value.status == hb.HB_ERR_INVALID_ARG
    for bad in (-0.1, 1.0, float("nan")):
        with pytest.raises(hb.HbError) as e:
            hb.hb_set_learned_min_saving(ctx, bad)
        assert e.value.status == hb.HB_ERR_INVALID_ARG
    hb.hb_set_sparse_rows(ctx, 0)
    hb.hb_set_learned_min_saving(ctx, 0.0)


@pytest.mark.parametrize("sparse", [1, 32])
def test_sparse_threshold_extremes(hb, ctx, sparse):
    """The per-lane form at its extremes (one live row per lane; up to 32):
    bit-exact against the oracle on the two-key recipe."""
    show(ctx, f"per-lane threshold {sparse}")
    if "two_keys_20k" not in _ORACLE:
        rel, rules = workloads.learned_10m(n=20_000)
        _ORACLE["two_keys_20k"] = (rel, rules, oracle.blocking(rel, rules, threads=8))
    rel, rules, want = _ORACLE["two_keys_20k"]
    hb.hb_set_sparse_rows(ctx, sparse)
    try:
        got, _ = run(hb, ctx, rel, rules, "heuristic")
    finally:
        hb.hb_set_sparse_rows(ctx, 0)
    assert np.array_equal(got, want)

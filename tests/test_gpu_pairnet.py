"""GPU parity of the per-pair cost network path (Section 4.2, "Evaluation
cost", "Estimated cost") against the oracle:

  * hb_pair_log_collect: the sampled pairs equal the oracle's sampler, the
    16 features equal the oracle's encoding exactly, and the "satisfied"
    label equals the oracle's predicate check on every sampled pair;
  * HB_COST_PAIR_NET: the costs compile writes equal norm(sum of the
    network's estimates) computed by the oracle from the network's outputs
    on the logged features (the only freedom is the order of an fp64 sum);
  * every plan built on those costs gives the oracle's matched pairs;
  * refused calls."""
import math
import os

import numpy as np
import pytest

import oracle
from gen import CATEGORICAL, ED, EQ, EQ_CROSS, JACCARD, ABSDIFF, Pred, Relation, int_column, string_column
from gen import workloads
from oracle import pairnet

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


def show(case):
    print(f"[gpu-case] pair network: {case}", flush=True)


def distinct(rules):
    """The rule set's distinct predicates in first-appearance order, with
    Jaccard thresholds in lowest terms (as the library keeps them)."""
    out, seen = [], set()
    for rule in rules:
        for p in rule:
            num, den = p.num, p.den
            if p.op == JACCARD:
                g = math.gcd(num, den)
                num, den = num // g, den // g
            key = (p.op, p.attr, p.k if p.op == ED else 0, p.q if p.op == JACCARD else 0,
                   num if p.op == JACCARD else 0, den if p.op == JACCARD else 1, p.d if p.op == ABSDIFF else 0)
            if key not in seen:
                seen.add(key)
                out.append(p)
    return out


def compiled(hb, ctx, rel, rules):
    rid = hb.hb_load_relation(ctx, rel.columns, rel.n_rows)
    rs = hb.hb_compile_rules(ctx, rid, rules)
    return rid, rs


def check_log(hb, ctx, rel, rules, samples, seed):
    rid, rs = compiled(hb, ctx, rel, rules)
    log = hb.hb_pair_log_collect(ctx, rid, rs, samples, seed)
    preds = distinct(rules)
    assert log["features"].shape == (len(preds) * samples, 16)
    want_pairs = [pairnet.sample_pair(seed, s, rel.n_rows) for s in range(samples)]
    assert [tuple(int(v) for v in p) for p in log["pairs"]] == want_pairs
    want_x = pairnet.sample_features(rel, preds, samples, seed)
    assert np.array_equal(log["features"], want_x)
    sat = log["labels"][:, 0].reshape(len(preds), samples)
    packed = np.array([(i << 32) | j for i, j in want_pairs], dtype=np.uint64)
    for x, p in enumerate(preds):
        # the predicate alone as a one-predicate rule, on every sampled pair
        want = oracle.eval_pairs(rel, [[p]], packed)
        assert np.array_equal(sat[x], want.astype(np.float32)), p
    cyc = log["labels"][:, 1]
    assert np.all(np.isfinite(cyc)) and np.all(cyc >= 0) and np.any(cyc > 0)
    hb.hb_release_relation(ctx, rid)
    return log


@pytest.mark.parametrize("seed", range(4))
def test_pair_log_matches_oracle(hb, ctx, seed):
    """Boundary string lengths (0, 1, q - 1, 31-33, 63-65, 127-129, 200),
    missing values, every predicate kind."""
    show(f"log, random_small seed {seed}")
    rel, rules = workloads.random_small(700 + seed, n=250, n_rules=6, null_p=0.1)
    check_log(hb, ctx, rel, rules, 300, 0x5EED + seed)


def test_pair_log_hand_relation(hb, ctx):
    show("log, hand relation")
    strings = [b"abcab", b"ab", None, b"x", b"a" * 40, b"ab", b"a" * 64, b"b" * 128, b""]
    ints = [5, 7, None, 5, 1, 2, 3, 4, 5]
    rel = Relation([string_column("s", strings), int_column("k", ints, CATEGORICAL),
                    int_column("i", [1, 2, 3, None, 5, 6, 7, 8, 9])], 9)
    rules = [[Pred(EQ, 1), Pred(ED, 0, k=3)], [Pred(EQ, 1), Pred(JACCARD, 0, q=2, num=2, den=4)],
             [Pred(EQ, 1), Pred(EQ, 0), Pred(ABSDIFF, 2, d=2)], [Pred(EQ, 1), Pred(JACCARD, 0, q=3, num=1, den=3)]]
    check_log(hb, ctx, rel, rules, 500, 11)


def train_pair_model(hb, ctx):
    """The per-pair model trained on logs of two relations."""
    xs, ts = [], []
    for k, (rel, rules) in enumerate((workloads.random_small(41, n=300, n_rules=8),
                                      workloads.plain_1m(n=20_000))):
        rid, rs = compiled(hb, ctx, rel, rules)
        log = hb.hb_pair_log_collect(ctx, rid, rs, 2048, 100 + k)
        hb.hb_release_relation(ctx, rid)
        xs.append(log["features"])
        ts.append(log["labels"])
    x, t = np.concatenate(xs), np.concatenate(ts)
    perm = np.random.default_rng(1).permutation(len(x))
    hb.hb_costmodel_select(ctx, "pair")
    try:
        hb.hb_costmodel_init(ctx, 5)
        loss = hb.hb_costmodel_train(ctx, x[perm], t[perm], epochs=20, batch=256, lr=2e-3)
    finally:
        hb.hb_costmodel_select(ctx, "block")
    return loss


def test_estimated_costs(hb, ctx):
    show("estimated costs")
    assert np.isfinite(train_pair_model(hb, ctx))
    for seed, (rel, rules) in enumerate((workloads.random_small(77, n=300, n_rules=7),
                                         workloads.plain_1m(n=20_000))):
        samples, cseed = 700 + 300 * seed, 0xC057 + seed
        rid, rs = compiled(hb, ctx, rel, rules)
        _, static = hb.hb_ruleset_estimates(ctx, rs)
        x = hb.hb_pair_log_collect(ctx, rid, rs, samples, cseed)["features"]
        hb.hb_costmodel_select(ctx, "pair")
        y = hb.hb_costmodel_predict(ctx, x)
        # the network's outputs, against the oracle's bf16 forward pass
        # (operands rounded alike; a hidden activation may round to the
        # neighbouring bf16 value, hence the loose bound)
        params = hb.hb_costmodel_get_params(ctx)
        hb.hb_costmodel_select(ctx, "block")
        want_y = pairnet.bf16_forward(unflat(params), x[:200].astype(np.float64))
        assert np.max(np.abs(y[:200] - want_y)) < 2e-2
        hb.hb_release_relation(ctx, rid)

        hb.hb_set_cost_estimate(ctx, "pair_net", samples, cseed)
        try:
            rid, rs = compiled(hb, ctx, rel, rules)
        finally:
            hb.hb_set_cost_estimate(ctx, "static")
        sp, cost = hb.hb_ruleset_estimates(ctx, rs)
        want = pairnet.estimated_costs(y, len(distinct(rules)), samples)
        assert np.allclose(cost, want, rtol=1e-9, atol=0), (cost, want)
        assert np.all(cost > 0) and np.all(cost <= 1) and cost.max() == 1.0
        hb.hb_release_relation(ctx, rid)
        # the selectivity estimate does not depend on the cost source
        rid, rs = compiled(hb, ctx, rel, rules)
        sp2, cost2 = hb.hb_ruleset_estimates(ctx, rs)
        assert np.array_equal(sp, sp2) and np.array_equal(cost2, static)
        hb.hb_release_relation(ctx, rid)


def unflat(v):
    p, o = {}, 0
    for k, s in (("W1", (16, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 2)), ("b3", (2,))):
        n = int(np.prod(s))
        p[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(s)
        o += n
    return p


@pytest.mark.parametrize("seed", range(4))
def test_plans_on_pair_costs_match_oracle(hb, ctx, seed):
    """Costs order predicates only: every plan built on the network's
    estimate returns the oracle's pairs."""
    show(f"plans on estimated costs, seed {seed}")
    if not _trained(hb, ctx):
        train_pair_model(hb, ctx)
    rel, rules = workloads.random_small(900 + seed, n=300 if seed % 2 else 120, n_rules=3 + seed)
    want = oracle.blocking(rel, rules, threads=8)
    hb.hb_set_cost_estimate(ctx, "pair_net", 512, seed)
    try:
        rid, rs = compiled(hb, ctx, rel, rules)
        hb.hb_partition(ctx, rid, rs)
        for plan in ("heuristic", "cheapest", "selective", "random_preds"):
            assert np.array_equal(hb.hb_match(ctx, rid, rs, plan), want), plan
        hb.hb_release_relation(ctx, rid)
    finally:
        hb.hb_set_cost_estimate(ctx, "static")


def test_two_keys_on_pair_costs(hb, ctx):
    show("two keys, 40k tuples, estimated costs")
    if not _trained(hb, ctx):
        train_pair_model(hb, ctx)
    rel, rules = workloads.learned_10m(n=40_000)
    want = oracle.blocking(rel, rules, threads=16)
    hb.hb_set_cost_estimate(ctx, "pair_net", 2048, 3)
    try:
        rid, rs = compiled(hb, ctx, rel, rules)
        _, cost = hb.hb_ruleset_estimates(ctx, rs)
        assert cost.max() == 1.0 and cost.min() > 0
        hb.hb_partition(ctx, rid, rs)
        assert np.array_equal(hb.hb_match(ctx, rid, rs, "heuristic"), want)
        hb.hb_release_relation(ctx, rid)
    finally:
        hb.hb_set_cost_estimate(ctx, "static")


def _trained(hb, ctx):
    hb.hb_costmodel_select(ctx, "pair")
    try:
        hb.hb_costmodel_get_params(ctx)
        return True
    except hb.HbError:
        return False
    finally:
        hb.hb_costmodel_select(ctx, "block")


def test_refused_and_degenerate(hb, ctx, tmp_path):
    show("refused calls")
    bad = lambda e: e.value.status == hb.HB_ERR_INVALID_ARG
    with pytest.raises(hb.HbError) as e:
        hb.hb_costmodel_select(ctx, 2)
    assert bad(e)
    for src, n in ((2, 16), ("pair_net", 0), ("pair_net", 65537)):
        with pytest.raises(hb.HbError) as e:
            hb.hb_set_cost_estimate(ctx, src, n, 1)
        assert bad(e)
    rel = Relation([int_column("k", [1, 1, 2, 1], CATEGORICAL), int_column("b", [1, 2, 3, 4], CATEGORICAL)], 4)
    # a fresh context has no per-pair model
    c2 = hb.hb_create(0, allocator="torch")
    try:
        hb.hb_set_cost_estimate(c2, "pair_net", 16, 1)
        rid = hb.hb_load_relation(c2, rel.columns, rel.n_rows)
        with pytest.raises(hb.HbError) as e:
            hb.hb_compile_rules(c2, rid, [[Pred(EQ, 0)]])
        assert e.value.status == hb.HB_ERR_STATE
    finally:
        c2.close()
    if not _trained(hb, ctx):
        train_pair_model(hb, ctx)
    rid = hb.hb_load_relation(ctx, rel.columns, rel.n_rows)
    ordered_rules = [[Pred(EQ, 0), Pred(EQ_CROSS, 0, attr_b=1)]]
    rs = hb.hb_compile_rules(ctx, rid, ordered_rules)
    with pytest.raises(hb.HbError) as e:
        hb.hb_pair_log_collect(ctx, rid, rs, 8, 1)
    assert bad(e)
    for n in (0, 65537):
        with pytest.raises(hb.HbError) as e:
            hb.hb_pair_log_collect(ctx, rid, hb.hb_compile_rules(ctx, rid, [[Pred(EQ, 0)]]), n, 1)
        assert bad(e)
    hb.hb_set_cost_estimate(ctx, "pair_net", 16, 1)
    try:
        with pytest.raises(hb.HbError) as e:
            hb.hb_compile_rules(ctx, rid, ordered_rules)
        assert bad(e)
    finally:
        hb.hb_set_cost_estimate(ctx, "static")
    hb.hb_release_relation(ctx, rid)
    # one tuple: no pairs, no log rows, every cost 1
    one = Relation([int_column("k", [1], CATEGORICAL), string_column("s", [b"abc"])], 1)
    rid = hb.hb_load_relation(ctx, one.columns, 1)
    rules = [[Pred(EQ, 0), Pred(ED, 1, k=1)]]
    assert hb.hb_pair_log_collect(ctx, rid, hb.hb_compile_rules(ctx, rid, rules), 8, 1)["features"].shape == (0, 16)
    hb.hb_set_cost_estimate(ctx, "pair_net", 16, 1)
    try:
        rs = hb.hb_compile_rules(ctx, rid, rules)
    finally:
        hb.hb_set_cost_estimate(ctx, "static")
    assert list(hb.hb_ruleset_estimates(ctx, rs)[1]) == [1.0, 1.0]
    hb.hb_release_relation(ctx, rid)
    # model files record which model they hold
    path = str(tmp_path / "pair.hbcm")
    hb.hb_costmodel_select(ctx, "pair")
    try:
        hb.hb_costmodel_save(ctx, path)
        hb.hb_costmodel_load(ctx, path)
    finally:
        hb.hb_costmodel_select(ctx, "block")
    with pytest.raises(hb.HbError) as e:
        hb.hb_costmodel_load(ctx, path)
    assert bad(e)
    assert os.path.getsize(path) == 8 + 24 + 4 * hb.HB_MLP_PARAMS + 8

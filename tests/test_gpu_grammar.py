"""GPU parity of the predicates t.A = c, s.A = c, t.A = s.B and t.A ~ s.B
(edit distance and q-gram Jaccard): libhb's ordered listing of Ca, through the C ABI, is
bit-exact against the oracle's, for every non-learned plan, across tiles and
their diagonals, with two keys, and with edit-distance patterns past 64
bytes.  Calls the ordered path does not take are refused."""
import numpy as np
import pytest

import oracle
from gen import (CATEGORICAL, CONTAIN, ED, ED_CROSS, EQ, EQ_CONST, EQ_CROSS, INT64, JACCARD, JACCARD_CROSS,
                 Pred, Relation, int_column, string_column)
from test_oracle_grammar import KEY, hand_relation, random_relation, random_rules

pytestmark = pytest.mark.gpu

PLANS = ["given", "heuristic", "cheapest", "selective", "random_preds", "random_rules"]


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
    print(f"[gpu-case] {case}", flush=True)


def match_all(hb, ctx, rel, rules, plans):
    rid = hb.hb_load_relation(ctx, rel.columns, rel.n_rows)
    rs = hb.hb_compile_rules(ctx, rid, rules)
    hb.hb_partition(ctx, rid, rs)
    outs = {p: hb.hb_match(ctx, rid, rs, p) for p in plans}
    hb.hb_release_relation(ctx, rid)
    return outs


def check(hb, ctx, rel, rules, plans=PLANS):
    want = oracle.blocking(rel, rules, threads=8)
    for plan, got in match_all(hb, ctx, rel, rules, plans).items():
        assert np.array_equal(got, want), (plan, len(got), len(want))
    return want


def test_hand_worked(hb, ctx):
    show("grammar: hand-worked relation")
    rel = hand_relation()
    for rules in ([[KEY, Pred(EQ_CONST, 1, side=0, c=1)]],
                  [[KEY, Pred(EQ_CONST, 2, side=1, c=1)]],
                  [[KEY, Pred(EQ_CROSS, 1, attr_b=2)]],
                  [[KEY, Pred(EQ_CONST, 2, side=1, c=1)], [KEY, Pred(EQ, 1)]],
                  [[KEY, Pred(EQ_CROSS, 1, attr_b=1)]]):
        check(hb, ctx, rel, rules)


@pytest.mark.parametrize("seed", range(10))
def test_random_small(hb, ctx, seed):
    show(f"grammar: random seed {seed}")
    check(hb, ctx, random_relation(seed, n=200), random_rules(seed))


@pytest.mark.parametrize("seed", range(4))
def test_several_tiles(hb, ctx, seed):
    # blocks of ~250 rows: 4 x 4 tile triangles with ragged edges and diagonals
    show(f"grammar: several tiles, seed {seed}")
    rel = random_relation(50 + seed, n=2000, n_keys=8)
    rules = random_rules(50 + seed)
    if not oracle.ordered(rules):
        rules = rules + [[KEY, Pred(EQ_CONST, 1, side=1, c=2)]]
    want = check(hb, ctx, rel, rules)
    assert len(want) > 0


def test_cross_edit_distance_short_strings(hb, ctx):
    # both valuations of t.s ~ s.u over short strings (empty and missing
    # values included), with and without a constant beside
    show("grammar: cross edit distance")
    rel = random_relation(77, n=1200, n_keys=5)
    for rules in ([[KEY, Pred(ED_CROSS, 4, attr_b=5, k=1)]],
                  [[KEY, Pred(ED_CROSS, 5, attr_b=4, k=2), Pred(EQ_CONST, 1, side=0, c=2)],
                   [KEY, Pred(ED, 4, k=0), Pred(EQ_CROSS, 2, attr_b=3)]]):
        assert len(check(hb, ctx, rel, rules)) > 0


def test_cross_jaccard(hb, ctx):
    """Both valuations of t.A ~ s.B under q-gram Jaccard: short strings with
    empty and missing values (random_relation), then two word-like string
    attributes of 5-40 bytes drawn from one alphabet so that many pairs are
    close, q = 1..3, beside a constant and a plain Jaccard."""
    show("grammar: cross Jaccard")
    rel = random_relation(78, n=1200, n_keys=5)
    for rules in ([[KEY, Pred(JACCARD_CROSS, 4, attr_b=5, q=1, num=1, den=2)]],
                  [[KEY, Pred(JACCARD_CROSS, 5, attr_b=4, q=2, num=1, den=3), Pred(EQ_CONST, 1, side=0, c=2)],
                   [KEY, Pred(JACCARD, 4, q=1, num=2, den=3)]]):
        assert len(check(hb, ctx, rel, rules)) > 0
    r = np.random.default_rng(79)
    n = 3000
    words = [bytes(r.integers(97, 103, size=int(r.integers(3, 8))).astype(np.uint8)) for _ in range(60)]

    def phrase():
        return b" ".join(words[int(w)] for w in r.integers(0, len(words), size=int(r.integers(1, 6))))[:40]
    a = [phrase() for _ in range(n)]
    b = [x if r.random() < 0.3 else phrase() for x in a]
    rel2 = Relation([int_column("k", [int(v) for v in r.integers(0, 40, size=n)], CATEGORICAL),
                     string_column("a", a), string_column("b", b)], n)
    for q, num, den in ((2, 1, 2), (3, 7, 10), (1, 4, 5)):
        rules = [[Pred(EQ, 0), Pred(JACCARD_CROSS, 1, attr_b=2, q=q, num=num, den=den)]]
        assert len(check(hb, ctx, rel2, rules, plans=["heuristic", "given"])) > 0
    # the asymmetric measure: containment of t's grams in s's, across the
    # two attributes and within one (ordered either way), alone and beside
    # a symmetric Jaccard rule
    for rules in ([[Pred(EQ, 0), Pred(CONTAIN, 1, attr_b=2, q=2, num=4, den=5)]],
                  [[Pred(EQ, 0), Pred(CONTAIN, 1, attr_b=1, q=3, num=1, den=1)]],
                  [[Pred(EQ, 0), Pred(CONTAIN, 2, attr_b=1, q=1, num=9, den=10)],
                   [Pred(EQ, 0), Pred(JACCARD, 1, q=2, num=1, den=2)]]):
        assert len(check(hb, ctx, rel2, rules, plans=["heuristic", "given"])) > 0
    for rules in ([[KEY, Pred(CONTAIN, 4, attr_b=5, q=1, num=2, den=3)]],
                  [[KEY, Pred(CONTAIN, 5, attr_b=5, q=2, num=1, den=2), Pred(EQ_CONST, 1, side=1, c=1)]]):
        assert len(check(hb, ctx, rel, rules)) > 0


def test_two_keys(hb, ctx):
    # a pair sharing both keys is evaluated in the first key's partition only
    show("grammar: two keys")
    r = np.random.default_rng(11)
    n = 1500
    k1 = int_column("k1", [int(x) for x in r.integers(0, 6, size=n)], CATEGORICAL)
    k2 = int_column("k2", [int(x) for x in r.integers(0, 5, size=n)], INT64)
    a = int_column("a", [int(x) for x in r.integers(0, 3, size=n)], CATEGORICAL)
    b = int_column("b", [int(x) for x in r.integers(0, 3, size=n)], INT64)
    rel = Relation([k1, k2, a, b], n)
    rules = [[Pred(EQ, 0), Pred(EQ_CROSS, 2, attr_b=3), Pred(EQ_CONST, 3, side=0, c=1)],
             [Pred(EQ, 1), Pred(EQ_CONST, 2, side=1, c=0)],
             [Pred(EQ, 1), Pred(EQ, 2), Pred(EQ, 3)]]
    check(hb, ctx, rel, rules)


def test_long_edit_distance_patterns(hb, ctx):
    # strings past 64 bytes take the register-state Myers kernel
    show("grammar: long edit-distance patterns")
    r = np.random.default_rng(5)
    n = 600
    base = [bytes(r.integers(97, 100, size=int(r.integers(60, 140))).astype(np.uint8)) for _ in range(n // 2)]
    strings = []
    for s in base:
        strings.append(s)
        t = bytearray(s)
        for _ in range(int(r.integers(0, 4))):
            t[int(r.integers(0, len(t)))] = int(r.integers(97, 100))
        strings.append(bytes(t))
    # a second string column: each row's string with 0-5 substitutions, or
    # a short unrelated one
    other = []
    for s in strings:
        t = bytearray(s)
        for _ in range(int(r.integers(0, 6))):
            t[int(r.integers(0, len(t)))] = int(r.integers(97, 100))
        other.append(bytes(t) if r.random() < 0.8 else bytes(r.integers(97, 100, size=5).astype(np.uint8)))
    rel = Relation([int_column("k", [int(x) for x in r.integers(0, 4, size=n)], CATEGORICAL),
                    string_column("s", strings),
                    int_column("a", [int(x) for x in r.integers(0, 2, size=n)], CATEGORICAL),
                    string_column("o", other)], n)
    for rules in ([[Pred(EQ, 0), Pred(EQ_CONST, 2, side=0, c=1), Pred(ED, 1, k=3)]],
                  [[Pred(EQ, 0), Pred(ED_CROSS, 1, attr_b=3, k=4)]],
                  [[Pred(EQ, 0), Pred(ED_CROSS, 3, attr_b=1, k=2), Pred(EQ_CONST, 2, side=1, c=0)],
                   [Pred(EQ, 0), Pred(ED, 3, k=1)]]):
        want = check(hb, ctx, rel, rules, plans=["given", "heuristic"])
        assert len(want) > 0


def test_refused_calls(hb, ctx):
    show("grammar: refused calls")
    rel = hand_relation()
    rid = hb.hb_load_relation(ctx, rel.columns, rel.n_rows)
    rs = hb.hb_compile_rules(ctx, rid, [[KEY, Pred(EQ_CONST, 1, side=0, c=1)]])
    hb.hb_partition(ctx, rid, rs)
    for call in (lambda: hb.hb_match(ctx, rid, rs, "learned"),
                 lambda: hb.hb_match_work(ctx, rid, rs, "heuristic"),
                 lambda: hb.hb_batch_create(ctx, [(rid, rs)], "heuristic", graph=False)):
        with pytest.raises(hb.HbError) as e:
            call()
        assert e.value.status == hb.HB_ERR_INVALID_ARG
    s = string_column("s", [b"x"] * rel.n_rows)
    rid2 = hb.hb_load_relation(ctx, rel.columns + [s], rel.n_rows)
    for rule, status in (([KEY, Pred(EQ_CONST, 3, side=0, c=1)], hb.HB_ERR_TYPE),     # constant on a string
                         ([KEY, Pred(EQ_CROSS, 1, attr_b=3)], hb.HB_ERR_TYPE),        # B is a string
                         ([KEY, Pred(EQ_CROSS, 1, attr_b=9)], hb.HB_ERR_INVALID_ARG),
                         ([KEY, Pred(EQ_CONST, 1, side=2, c=1)], hb.HB_ERR_INVALID_ARG),
                         ([KEY, Pred(ED_CROSS, 1, attr_b=3, k=1)], hb.HB_ERR_TYPE),     # A is an int
                         ([KEY, Pred(ED_CROSS, 3, attr_b=3, k=300)], hb.HB_ERR_INVALID_ARG),
                         ([KEY, Pred(JACCARD_CROSS, 1, attr_b=3, q=2, num=1, den=2)], hb.HB_ERR_TYPE),
                         ([KEY, Pred(JACCARD_CROSS, 3, attr_b=3, q=9, num=1, den=2)], hb.HB_ERR_INVALID_ARG),
                         ([KEY, Pred(CONTAIN, 1, attr_b=3, q=2, num=1, den=2)], hb.HB_ERR_TYPE),
                         ([KEY, Pred(CONTAIN, 3, attr_b=3, q=2, num=3, den=2)], hb.HB_ERR_INVALID_ARG),
                         ([Pred(EQ_CROSS, 0, attr_b=0)], hb.HB_ERR_UNBLOCKABLE)):   # never a key
        with pytest.raises(hb.HbError) as e:
            hb.hb_compile_rules(ctx, rid2, [rule])
        assert e.value.status == status, rule
    # the plain path is unaffected: the same relation with a symmetric rule
    rs3 = hb.hb_compile_rules(ctx, rid, [[KEY, Pred(EQ, 1)]])
    hb.hb_partition(ctx, rid, rs3)
    assert np.array_equal(hb.hb_match(ctx, rid, rs3, "heuristic"), oracle.blocking(rel, [[KEY, Pred(EQ, 1)]]))
    hb.hb_release_relation(ctx, rid)
    hb.hb_release_relation(ctx, rid2)

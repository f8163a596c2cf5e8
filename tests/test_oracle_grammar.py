"""Pins of the oracle's predicates t.A = c, s.A = c, t.A = s.B and t.A ~ s.B
under edit distance and under q-gram Jaccard (Section 2, "Predicates" and
"Semantics") and of its ordered listing of Ca (CPU only).

A valuation binds t to the pair's first row and s to its second; a rule set
with a predicate that tells t from s lists every ordered pair whose valuation
has a witness.  The pins: a hand-worked relation, the transposition of t and
s, the reduction of t.A = s.A to equality, and the listing of a symmetric
rule set forced into ordered form.
"""
import numpy as np
import pytest

import oracle
from gen import (CATEGORICAL, CONTAIN, ED, ED_CROSS, EQ, EQ_CONST, EQ_CROSS, INT64, JACCARD, JACCARD_CROSS,
                 Pred, Relation, int_column, string_column)


def P(i, j):
    return (i << 32) | j


def pairs(*ps):
    return np.array(sorted(P(i, j) for i, j in ps), dtype=np.uint64)


def hand_relation():
    #  row  k  a     b
    #   0   1  1     2
    #   1   1  2     1
    #   2   1  1     1
    #   3   2  1     5
    #   4   2  -     1
    #   5   3  1     1     (alone in its block)
    k = int_column("k", [1, 1, 1, 2, 2, 3], CATEGORICAL)
    a = int_column("a", [1, 2, 1, 1, None, 1], CATEGORICAL)
    b = int_column("b", [2, 1, 1, 5, 1, 1], INT64)
    return Relation([k, a, b], 6)


KEY = Pred(EQ, 0)


def test_hand_worked_constant_on_t():
    # t.a = 1: blocks {0, 1, 2} and {3, 4}; t ranges over rows with a = 1
    # (0, 2, 3); row 4's a is missing, so (4, 3) fails
    got = oracle.blocking(hand_relation(), [[KEY, Pred(EQ_CONST, 1, side=0, c=1)]])
    assert np.array_equal(got, pairs((0, 1), (0, 2), (2, 0), (2, 1), (3, 4)))


def test_hand_worked_constant_on_s():
    # s.b = 1: s ranges over rows 1, 2 (block 1) and 4 (block 2)
    got = oracle.blocking(hand_relation(), [[KEY, Pred(EQ_CONST, 2, side=1, c=1)]])
    assert np.array_equal(got, pairs((0, 1), (0, 2), (1, 2), (2, 1), (3, 4)))


def test_hand_worked_cross_attribute():
    # t.a = s.b inside each block:
    #   (0,1): a0=1 b1=1 yes   (0,2): a0=1 b2=1 yes   (1,0): a1=2 b0=2 yes
    #   (1,2): a1=2 b2=1 no    (2,0): a2=1 b0=2 no    (2,1): a2=1 b1=1 yes
    #   (3,4): a3=1 b4=1 yes   (4,3): a4 missing  no
    got = oracle.blocking(hand_relation(), [[KEY, Pred(EQ_CROSS, 1, attr_b=2)]])
    assert np.array_equal(got, pairs((0, 1), (0, 2), (1, 0), (2, 1), (3, 4)))


def test_hand_worked_mixed_rule_set():
    # s.b = 1 (above) or a = a (rows 0 and 2 only; row 4's a is missing):
    # the symmetric rule's pair appears in both orders
    got = oracle.blocking(hand_relation(), [[KEY, Pred(EQ_CONST, 2, side=1, c=1)], [KEY, Pred(EQ, 1)]])
    assert np.array_equal(got, pairs((0, 1), (0, 2), (1, 2), (2, 0), (2, 1), (3, 4)))


def test_hand_worked_cross_edit_distance():
    #  row  k  x      y
    #   0   1  abc    abd
    #   1   1  xyz    abc
    #   2   1  abd    -
    # ED(t.x, s.y): (0,1) abc/abc 0; (0,2) y missing; (1,0) xyz/abd 3;
    # (1,2) y missing; (2,0) abd/abd 0; (2,1) abd/abc 1
    rel = Relation([int_column("k", [1, 1, 1], CATEGORICAL), string_column("x", [b"abc", b"xyz", b"abd"]),
                    string_column("y", [b"abd", b"abc", None])], 3)
    got0 = oracle.blocking(rel, [[KEY, Pred(ED_CROSS, 1, attr_b=2, k=0)]])
    assert np.array_equal(got0, pairs((0, 1), (2, 0)))
    got1 = oracle.blocking(rel, [[KEY, Pred(ED_CROSS, 1, attr_b=2, k=1)]])
    assert np.array_equal(got1, pairs((0, 1), (2, 0), (2, 1)))
    got3 = oracle.blocking(rel, [[KEY, Pred(ED_CROSS, 1, attr_b=2, k=3)]])
    assert np.array_equal(got3, pairs((0, 1), (1, 0), (2, 0), (2, 1)))


def test_hand_worked_cross_jaccard():
    #  row  k  x      y
    #   0   1  abcd   bcde
    #   1   1  bcd    abcd
    #   2   1  xy     -
    # 2-gram sets: x0 {ab,bc,cd}  x1 {bc,cd}  x2 {xy};  y0 {bc,cd,de}  y1 {ab,bc,cd}
    # J(t.x, s.y):
    #   (0,1) x0/y1 = 3/3 = 1      (1,0) x1/y0 = 2/3      (2,0) x2/y0 = 0/4
    #   (2,1) x2/y1 = 0/4          (0,2), (1,2): y2 missing
    rel = Relation([int_column("k", [1, 1, 1], CATEGORICAL), string_column("x", [b"abcd", b"bcd", b"xy"]),
                    string_column("y", [b"bcde", b"abcd", None])], 3)
    got_half = oracle.blocking(rel, [[KEY, Pred(JACCARD_CROSS, 1, attr_b=2, q=2, num=1, den=2)]])
    assert np.array_equal(got_half, pairs((0, 1), (1, 0)))
    got_two_thirds = oracle.blocking(rel, [[KEY, Pred(JACCARD_CROSS, 1, attr_b=2, q=2, num=2, den=3)]])
    assert np.array_equal(got_two_thirds, pairs((0, 1), (1, 0)))
    got_high = oracle.blocking(rel, [[KEY, Pred(JACCARD_CROSS, 1, attr_b=2, q=2, num=7, den=10)]])
    assert np.array_equal(got_high, pairs((0, 1)))
    got_zero = oracle.blocking(rel, [[KEY, Pred(JACCARD_CROSS, 1, attr_b=2, q=2, num=0, den=1)]])
    assert np.array_equal(got_zero, pairs((0, 1), (1, 0), (2, 0), (2, 1)))


def test_hand_worked_containment():
    #  row  k  x     y
    #   0   1  ab    abc
    #   1   1  abc   ab
    #   2   1  ""    bcz
    # 2-gram sets: x0 {ab}  x1 {ab,bc}  x2 {};  y0 {ab,bc}  y1 {ab}  y2 {bc,cz}
    # share of t.x's grams in s.y's:
    #   (0,1) 1/1  (0,2) 0/1  (1,0) 2/2  (1,2) 1/2  (2,0) 0/0  (2,1) 0/0 (an
    #   empty set is contained in anything)
    rel = Relation([int_column("k", [1, 1, 1], CATEGORICAL), string_column("x", [b"ab", b"abc", b""]),
                    string_column("y", [b"abc", b"ab", b"bcz"])], 3)
    full = oracle.blocking(rel, [[KEY, Pred(CONTAIN, 1, attr_b=2, q=2, num=1, den=1)]])
    assert np.array_equal(full, pairs((0, 1), (1, 0), (2, 0), (2, 1)))
    half = oracle.blocking(rel, [[KEY, Pred(CONTAIN, 1, attr_b=2, q=2, num=1, den=2)]])
    assert np.array_equal(half, pairs((0, 1), (1, 0), (1, 2), (2, 0), (2, 1)))
    # on one attribute the measure stays asymmetric: x0 in x1 is 1, x1 in x0 is 1/2
    same = oracle.blocking(rel, [[KEY, Pred(CONTAIN, 1, attr_b=1, q=2, num=1, den=1)]])
    assert np.array_equal(same, pairs((0, 1), (2, 0), (2, 1)))
    same_half = oracle.blocking(rel, [[KEY, Pred(CONTAIN, 1, attr_b=1, q=2, num=1, den=2)]])
    assert np.array_equal(same_half, pairs((0, 1), (1, 0), (2, 0), (2, 1)))


@pytest.mark.parametrize("seed", range(6))
def test_jaccard_implies_containment(seed):
    # |A & B| / |A| >= |A & B| / |A | B|: every pair whose Jaccard reaches the
    # threshold is contained to it, in both orders
    rel = random_relation(400 + seed)
    for q, num, den in ((1, 1, 2), (2, 1, 3), (2, 2, 3)):
        jac = oracle.blocking(rel, [[KEY, Pred(JACCARD, 4, q=q, num=num, den=den)]])
        both = set(jac.tolist()) | set(transpose_pairs(jac).tolist())
        cont = set(oracle.blocking(rel, [[KEY, Pred(CONTAIN, 4, attr_b=4, q=q, num=num, den=den)]]).tolist())
        assert both <= cont


def test_ordered_flag():
    assert not oracle.ordered([[KEY, Pred(EQ, 1)]])
    assert not oracle.ordered([[KEY, Pred(EQ_CROSS, 1, attr_b=1)]])
    assert oracle.ordered([[KEY, Pred(EQ_CROSS, 1, attr_b=2)]])
    assert oracle.ordered([[KEY], [KEY, Pred(EQ_CONST, 1, side=1, c=0)]])
    assert oracle.ordered([[KEY, Pred(ED_CROSS, 1, attr_b=2, k=1)]])
    assert not oracle.ordered([[KEY, Pred(ED_CROSS, 1, attr_b=1, k=1)]])
    assert oracle.ordered([[KEY, Pred(JACCARD_CROSS, 1, attr_b=2, q=2, num=1, den=2)]])
    assert not oracle.ordered([[KEY, Pred(JACCARD_CROSS, 1, attr_b=1, q=2, num=1, den=2)]])
    assert oracle.ordered([[KEY, Pred(CONTAIN, 1, attr_b=1, q=2, num=1, den=2)]])   # asymmetric


def random_relation(seed, n=160, n_keys=6, dom=4, p_missing=0.1):
    r = np.random.default_rng(seed)

    def vals(hi):
        v = r.integers(0, hi, size=n)
        return [None if r.random() < p_missing else int(x) for x in v]

    k = int_column("k", [int(x) for x in r.integers(0, n_keys, size=n)], CATEGORICAL)
    a = int_column("a", vals(dom), CATEGORICAL)
    b = int_column("b", vals(dom), INT64)
    c = int_column("c", vals(dom), INT64)
    s = string_column("s", [bytes(r.integers(97, 100, size=int(r.integers(1, 6))).astype(np.uint8))
                            for _ in range(n)])
    u = string_column("u", [None if r.random() < p_missing else
                            bytes(r.integers(97, 100, size=int(r.integers(0, 6))).astype(np.uint8))
                            for _ in range(n)])
    return Relation([k, a, b, c, s, u], n)


def random_rules(seed):
    """1-3 rules over the key, each with 1-3 of: a constant on t or s, a
    cross-attribute equality, a plain equality, an edit distance, an edit
    distance or a q-gram Jaccard across the two string attributes."""
    r = np.random.default_rng(seed)
    rules = []
    for _ in range(int(r.integers(1, 4))):
        rule = [KEY]
        for _ in range(int(r.integers(1, 4))):
            kind = int(r.integers(0, 6))
            if kind == 0:
                rule.append(Pred(EQ_CONST, int(r.integers(1, 4)), side=int(r.integers(0, 2)), c=int(r.integers(0, 4))))
            elif kind == 1:
                a, b = r.choice([1, 2, 3], size=2, replace=False)
                rule.append(Pred(EQ_CROSS, int(a), attr_b=int(b)))
            elif kind == 2:
                rule.append(Pred(EQ, int(r.integers(1, 4))))
            elif kind == 3:
                rule.append(Pred(ED, 4, k=int(r.integers(0, 3))))
            elif kind == 4:
                a = int(r.integers(4, 6))
                rule.append(Pred(ED_CROSS, a, attr_b=9 - a, k=int(r.integers(0, 3))))
            else:
                a = int(r.integers(4, 6))
                num, den = ((1, 3), (1, 2), (2, 3))[int(r.integers(0, 3))]
                rule.append(Pred(JACCARD_CROSS, a, attr_b=9 - a, q=int(r.integers(1, 3)), num=num, den=den))
        rules.append(rule)
    return rules


def transpose_pred(p):
    """The same predicate with t and s exchanged."""
    if p.op == EQ_CONST:
        return Pred(EQ_CONST, p.attr, side=1 - p.side, c=p.c)
    if p.op == EQ_CROSS:
        return Pred(EQ_CROSS, p.attr_b, attr_b=p.attr)
    if p.op == ED_CROSS:   # the distance is symmetric in its two strings
        return Pred(ED_CROSS, p.attr_b, attr_b=p.attr, k=p.k)
    if p.op == JACCARD_CROSS:   # so is the Jaccard similarity of two sets
        return Pred(JACCARD_CROSS, p.attr_b, attr_b=p.attr, q=p.q, num=p.num, den=p.den)
    return p


def transpose_pairs(x):
    return np.sort((x << np.uint64(32)) | (x >> np.uint64(32)))


@pytest.mark.parametrize("seed", range(12))
def test_exchanging_t_and_s_transposes_ca(seed):
    rel, rules = random_relation(seed), random_rules(seed)
    if not oracle.ordered(rules):
        rules = rules + [[KEY, Pred(EQ_CONST, 1, side=0, c=99)]]
    got = oracle.blocking(rel, rules)
    swapped = oracle.blocking(rel, [[transpose_pred(p) for p in rule] for rule in rules])
    assert np.array_equal(swapped, transpose_pairs(got))


@pytest.mark.parametrize("seed", range(6))
def test_cross_on_one_attribute_is_equality(seed):
    rel = random_relation(100 + seed)
    for a in (1, 2, 3):
        got = oracle.blocking(rel, [[KEY, Pred(EQ_CROSS, a, attr_b=a)]])
        want = oracle.blocking(rel, [[KEY, Pred(EQ, a)]])
        assert np.array_equal(got, want)
    for a in (4, 5):
        for k in (0, 2):
            got = oracle.blocking(rel, [[KEY, Pred(ED_CROSS, a, attr_b=a, k=k)]])
            assert np.array_equal(got, oracle.blocking(rel, [[KEY, Pred(ED, a, k=k)]]))
        for q, num, den in ((1, 1, 2), (2, 2, 3), (2, 0, 1)):
            got = oracle.blocking(rel, [[KEY, Pred(JACCARD_CROSS, a, attr_b=a, q=q, num=num, den=den)]])
            want = oracle.blocking(rel, [[KEY, Pred(JACCARD, a, q=q, num=num, den=den)]])
            assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(6))
def test_never_true_ordered_rule_only_relists(seed):
    # a constant no row holds makes the rule set ordered without adding a
    # witness: the result is the symmetric one, each pair in both orders
    rel = random_relation(200 + seed)
    sym = [[KEY, Pred(EQ, 1)], [KEY, Pred(ED, 4, k=1), Pred(EQ, 3)]]
    base = oracle.blocking(rel, sym)
    got = oracle.blocking(rel, sym + [[KEY, Pred(EQ_CONST, 2, side=0, c=12345)]])
    assert np.array_equal(got, np.sort(np.concatenate([base, transpose_pairs(base)])))


@pytest.mark.parametrize("seed", range(6))
def test_ordered_blocked_equals_full_and_eval(seed):
    rel, rules = random_relation(300 + seed, n=90), random_rules(300 + seed)
    got = oracle.blocking(rel, rules)
    assert np.array_equal(got, oracle.blocking(rel, rules, mode="full"))
    assert np.all(oracle.eval_pairs(rel, rules, got))
    if oracle.ordered(rules):
        # every pair not listed, in a block, fails its valuation
        listed = set(got.tolist())
        keys = rel.columns[0].values
        cand = [P(i, j) for i in range(rel.n_rows) for j in range(rel.n_rows)
                if i != j and keys[i] == keys[j] and P(i, j) not in listed]
        assert not np.any(oracle.eval_pairs(rel, rules, np.array(cand, dtype=np.uint64)))

"""Pins of the oracle's per-pair cost network pieces (Section 4.2,
"Evaluation cost", "Estimated cost"): the pair sampler against its exact
distribution, the 16 pair features against values worked out by hand from
their definition, and the estimated cost against a closed form through a
hand-built network whose estimate is 2^(L / 64) - 1 cycles."""
import math

import numpy as np
import pytest

from gen import ABSDIFF, CATEGORICAL, ED, EQ, EQ_CROSS, ED_CROSS, JACCARD, CONTAIN, Pred, Relation
from gen import int_column, string_column
from oracle import pairnet


def rel_small():
    strings = [b"abcab", b"ab", None, b"x", b"a" * 40, b"ab", b"a" * 64, b"b" * 128]
    ints = [5, 7, None, 5, 1, 2, 3, 4]
    return Relation([string_column("s", strings), int_column("k", ints, CATEGORICAL),
                     string_column("t", [b"q"] * 8)], 8)


def test_sampler_distribution():
    """On n = 3 tuples the sampler gives (i, i+1 mod n) with probability 2/9
    each and (i, i+2 mod n) with 1/9 each (j = i is moved to i + 1); never
    i = j; two seeds give different streams."""
    n, m = 3, 30000
    counts = np.zeros((n, n))
    for s in range(m):
        i, j = pairnet.sample_pair(12345, s, n)
        assert 0 <= i < n and 0 <= j < n and i != j
        counts[i, j] += 1
    for i in range(n):
        for d, p in ((1, 2 / 9), (2, 1 / 9)):
            sd = math.sqrt(m * p * (1 - p))
            assert abs(counts[i, (i + d) % n] - m * p) < 5 * sd, (i, d, counts)
    a = [pairnet.sample_pair(1, s, 1000) for s in range(50)]
    b = [pairnet.sample_pair(2, s, 1000) for s in range(50)]
    assert a != b
    # both members of a pair range over the whole relation
    big = [pairnet.sample_pair(7, s, 10) for s in range(2000)]
    assert {i for i, _ in big} == set(range(10)) and {j for _, j in big} == set(range(10))


def test_features_by_hand():
    rel = rel_small()
    f = lambda p, i, j: pairnet.pair_features(rel, p, i, j).tolist()
    jac = Pred(JACCARD, 0, q=2, num=1, den=2)
    # G_2("abcab") = {ab, bc, ca}, G_2("ab") = {ab}
    assert f(jac, 0, 1) == [0, 0, 0, 0, 1, 1, 1, 5 / 64, 2 / 64, 3 / 64, 1 / 64, 0, 0.5, 2 / 64, 3 / 64, 1]
    # "x" is shorter than q: one code, and the short flag
    assert f(jac, 0, 3) == [0, 0, 0, 0, 1, 1, 1, 5 / 64, 1 / 64, 3 / 64, 1 / 64, 1, 0.5, 1 / 64, 4 / 64, 1]
    # a missing value: absent, length and count 0
    assert f(jac, 0, 2) == [0, 0, 0, 0, 1, 1, 0, 5 / 64, 0, 3 / 64, 0, 0, 0.5, 0, 5 / 64, 1]
    third = pairnet.pair_features(rel, Pred(JACCARD, 0, q=3, num=1, den=3), 1, 0)
    assert third[12] == np.float32(1 / 3) and third[11] == 1 and third[9] == 1 / 64 and third[10] == 3 / 64
    ed = Pred(ED, 0, k=3)
    # pattern words: 40 bytes -> one 64-bit word; 5 bytes -> the 32-bit table (0)
    assert f(ed, 4, 0) == [0, 0, 0, 1, 0, 1, 1, 40 / 64, 5 / 64, 0.25, 3 / 16, 0, 0, 5 / 64, 35 / 64, 1]
    assert f(ed, 0, 4)[9] == 0 and f(ed, 7, 0)[9] == 2 / 4 and f(ed, 6, 0)[9] == 1 / 4
    eqs = Pred(EQ, 0)
    assert f(eqs, 1, 5) == [0, 0, 1, 0, 0, 1, 1, 2 / 64, 2 / 64, 1, 0, 0, 0, 2 / 64, 0, 1]
    assert f(eqs, 0, 1)[9] == 0 and f(eqs, 2, 2)[9] == 0
    # value predicates: kind, presence and the constant only
    assert f(Pred(EQ, 1), 0, 2) == [1, 0, 0, 0, 0, 1, 0] + [0] * 8 + [1]
    assert f(Pred(ABSDIFF, 1, d=2), 3, 0) == [0, 1, 0, 0, 0, 1, 1] + [0] * 8 + [1]
    # t.A = s.A and t.A ~ s.A written in the cross form are the plain kinds
    assert f(Pred(EQ_CROSS, 1, attr_b=1), 0, 1) == f(Pred(EQ, 1), 0, 1)
    assert f(Pred(ED_CROSS, 0, k=3, attr_b=0), 4, 0) == f(ed, 4, 0)
    for p in (Pred(EQ_CROSS, 1, attr_b=0), Pred(ED_CROSS, 0, k=1, attr_b=2),
              Pred(CONTAIN, 0, q=2, num=1, den=2, attr_b=0)):
        with pytest.raises(ValueError):
            pairnet.kind(rel, p)


def length_network(row_from=7, shift=16):
    """Hidden units 0..15 copy the features, the second output reads
    feature `row_from` / `shift`: y = L1 / (64 * 16) gives 2^(L1 / 64) - 1."""
    p = {"W1": np.zeros((16, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "W3": np.zeros((64, 2)), "b3": np.zeros(2)}
    for k in range(16):
        p["W1"][k, k] = 1.0
        p["W2"][k, k] = 1.0
    p["W3"][row_from, 1] = 1.0 / shift
    return p


def test_estimate_closed_form():
    """Lengths 64 and 128 estimate 1 and 3 cycles per pair: two predicates
    sampled only on such rows cost 1/3 and 1; sums are over the sample."""
    rel = Relation([string_column("a", [b"a" * 64, b"b" * 64]),
                    string_column("b", [b"c" * 128, b"d" * 128])], 2)
    preds = [Pred(ED, 0, k=1), Pred(ED, 1, k=1)]
    x = pairnet.sample_features(rel, preds, 5, 99)
    assert x.shape == (10, 16)
    y = pairnet.bf16_forward(length_network(), x)
    assert np.allclose(pairnet.pair_cycles(y), [1.0] * 5 + [3.0] * 5, rtol=0, atol=1e-12)
    assert pairnet.estimated_costs(y, 2, 5) == [1 / 3, 1.0]


def test_estimate_floor_clamp_and_degenerate():
    y = np.array([[0.0, -1.0], [0.0, 0.0], [0.0, 5.0], [0.0, 4.0]])
    c = pairnet.pair_cycles(y)
    assert c[0] == 0 and c[1] == 0 and c[2] == 2.0 ** 64 - 1 and c[3] == 2.0 ** 64 - 1
    # a predicate whose estimate is zero keeps the floor; the other is 1
    assert pairnet.estimated_costs(y, 2, 2) == [pairnet.COST_FLOOR, 1.0]
    assert pairnet.estimated_costs(np.zeros((4, 2)), 2, 2) == [1.0, 1.0]
    assert pairnet.estimated_costs(np.zeros((0, 2)), 3, 0) == [1.0, 1.0, 1.0]
    assert pairnet.estimated_costs(np.zeros((0, 2)), 0, 7) == []


def test_estimate_orders_by_length():
    """Through the length network, a longer attribute costs more: the
    estimate follows the sampled lengths of D x D, not a static type rule."""
    r = np.random.default_rng(3)
    short = [bytes(r.integers(97, 100, size=int(r.integers(1, 20))).astype(np.uint8)) for _ in range(50)]
    long_ = [bytes(r.integers(97, 100, size=int(r.integers(100, 200))).astype(np.uint8)) for _ in range(50)]
    rel = Relation([string_column("s", short), string_column("l", long_)], 50)
    preds = [Pred(ED, 0, k=2), Pred(ED, 1, k=2), Pred(EQ, 0)]
    x = pairnet.sample_features(rel, preds, 64, 5)
    costs = pairnet.estimated_costs(pairnet.bf16_forward(length_network(), x), 3, 64)
    assert costs[1] == 1.0 and costs[0] < 0.2 and costs[2] == costs[0]

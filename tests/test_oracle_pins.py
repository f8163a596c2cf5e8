"""Pins of the CPU oracle against facts fixed outside it (CPU only).

Edit distance: shortest paths in the graph of single-character edits (an
independent computation of the Levenshtein distance), closed forms.
Jaccard: closed forms on constructed strings, exact rational boundaries.
Semantics: Table 1 with Examples 3 and 9 (missing values), invariants
(symmetry, order and partition independence, monotonicity, union, exact
duplicates, blocked = full), closed-form candidate counts.
"""
import itertools
import json
import os
from collections import deque

import numpy as np
import pytest

import oracle
from gen import (ABSDIFF, CATEGORICAL, ED, EQ, INT64, JACCARD, Pred, Relation, int_column,
                 string_column)
from gen import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------- edit distance

def _all_strings(alphabet, max_len):
    out = []
    for L in range(max_len + 1):
        out.extend("".join(t) for t in itertools.product(alphabet, repeat=L))
    return out


def _edit_graph_distances(alphabet, max_len):
    """BFS over strings of length <= max_len where an edge is one insert,
    delete or substitute.  An optimal edit sequence can do its deletions,
    then substitutions, then insertions, so it never leaves this space."""
    nodes = _all_strings(alphabet, max_len)

    def nbrs(s):
        for x in range(len(s)):
            yield s[:x] + s[x + 1:]
            for c in alphabet:
                if c != s[x]:
                    yield s[:x] + c + s[x + 1:]
        if len(s) < max_len:
            for x in range(len(s) + 1):
                for c in alphabet:
                    yield s[:x] + c + s[x:]

    dist = {}
    for src in nodes:
        d = {src: 0}
        dq = deque([src])
        while dq:
            u = dq.popleft()
            for v in nbrs(u):
                if v not in d:
                    d[v] = d[u] + 1
                    dq.append(v)
        dist[src] = d
    return nodes, dist


@pytest.mark.parametrize("alphabet,max_len", [("ab", 6), ("abc", 4)])
def test_levenshtein_equals_edit_graph_shortest_path(alphabet, max_len):
    nodes, dist = _edit_graph_distances(alphabet, max_len)
    for a in nodes:
        for b in nodes:
            assert oracle.levenshtein(a.encode(), b.encode()) == dist[a][b], (a, b)


def test_levenshtein_closed_forms():
    assert oracle.levenshtein(b"kitten", b"sitting") == 3
    assert oracle.levenshtein(b"", b"") == 0
    rng = np.random.default_rng(7)
    for _ in range(200):
        m, n = rng.integers(0, 30, size=2)
        a = bytes(rng.integers(97, 101, size=m).astype(np.uint8))
        b = bytes(rng.integers(97, 101, size=n).astype(np.uint8))
        c = bytes(rng.integers(97, 101, size=rng.integers(0, 30)).astype(np.uint8))
        dab = oracle.levenshtein(a, b)
        assert oracle.levenshtein(a, a) == 0
        assert oracle.levenshtein(a, b"") == len(a)
        assert oracle.levenshtein(b"", b) == len(b)
        assert dab == oracle.levenshtein(b, a)
        assert abs(len(a) - len(b)) <= dab <= max(len(a), len(b))
        assert dab <= oracle.levenshtein(a, c) + oracle.levenshtein(c, b)
        if len(a):
            x = int(rng.integers(0, len(a)))
            sub = a[:x] + b"z" + a[x + 1:]
            assert oracle.levenshtein(a, sub) == 1
            assert oracle.levenshtein(a, a[:x] + a[x + 1:]) == 1


def test_levenshtein_long_boundaries():
    # lengths around machine-word multiples; distance of a string to its
    # prefix is the length difference, and one substitution costs 1
    base = bytes((97 + (i * 7) % 26) for i in range(260))
    for L in (63, 64, 65, 127, 128, 129, 200):
        s = base[:L]
        assert oracle.levenshtein(s, base[:L - 1]) == 1
        assert oracle.levenshtein(s, base[:L - 10]) == 10
        t = s[:L // 2] + b"#" + s[L // 2 + 1:]
        assert oracle.levenshtein(s, t) == 1
        assert oracle.levenshtein(s, b"") == L


# ------------------------------------------------------------------ jaccard

def test_qgram_set_sizes():
    # all windows distinct -> |G| = L - q + 1
    assert oracle.qgram_stats(b"abcdefgh", b"", 3)[0] == 6
    assert oracle.qgram_stats(b"aaaaa", b"", 3)[0] == 1
    assert oracle.qgram_stats(b"abab", b"", 2)[0] == 2        # {ab, ba}
    assert oracle.qgram_stats(b"ab", b"", 3)[0] == 1          # shorter than q -> {s}
    assert oracle.qgram_stats(b"", b"", 3)[0] == 0


def test_jaccard_closed_form_interior_substitution():
    # A 30-character string with distinct characters has G = 28 distinct
    # 3-grams; replacing one interior character by a new one replaces
    # exactly q = 3 grams by q new ones: I = G - q = 25, U = G + q = 31.
    s = bytes(range(65, 95))
    t = s[:15] + b"~" + s[16:]
    g, inter, uni = oracle.qgram_stats(s, t, 3)
    assert (g, inter, uni) == (28, 25, 31)
    assert oracle.jaccard_ge(s, t, 3, 25, 31)
    assert not oracle.jaccard_ge(s, t, 3, 13, 16)      # 13/16 > 25/31
    assert oracle.jaccard_ge(s, t, 3, 4, 5)            # 4/5 < 25/31


def test_jaccard_exact_rational_boundary():
    # q = 1: {a,b,c,d} vs {a,b,c,e}: I = 3, U = 5
    a, b = b"abcd", b"abce"
    assert oracle.qgram_stats(a, b, 1)[1:] == (3, 5)
    assert oracle.jaccard_ge(a, b, 1, 3, 5)
    assert oracle.jaccard_ge(a, b, 1, 6, 10)
    assert not oracle.jaccard_ge(a, b, 1, 601, 1000)
    assert oracle.jaccard_ge(a, b, 1, 599, 1000)
    assert not oracle.jaccard_ge(b"abcd", b"abef", 1, 3, 5)   # I = 2, U = 6


def test_jaccard_special_sets():
    assert oracle.jaccard_ge(b"hello world", b"hello world", 3, 1, 1)
    assert oracle.qgram_stats(b"abcabc", b"xyzxyz", 2)[1] == 0
    assert not oracle.jaccard_ge(b"abcabc", b"xyzxyz", 2, 1, 100)
    assert oracle.jaccard_ge(b"abcabc", b"xyzxyz", 2, 0, 1)       # theta = 0
    assert oracle.jaccard_ge(b"", b"", 3, 1, 1)                   # J(empty, empty) = 1
    assert not oracle.jaccard_ge(b"", b"abc", 3, 1, 100)
    assert oracle.qgram_stats(b"ab", b"ab", 3)[1:] == (1, 1)      # both shorter than q
    assert oracle.qgram_stats(b"ab", b"abc", 3)[1:] == (0, 2)


# ---------------------------------------------------------------- semantics

def _table1():
    with open(os.path.join(HERE, "golden", "table1_products.json")) as f:
        g = json.load(f)
    c = g["columns"]

    def codes(vals):
        d = {}
        return [None if v is None else d.setdefault(v, len(d)) for v in vals]

    cols = [
        string_column("pno", [s.encode() for s in c["pno"]]),
        string_column("pname", [s.encode() for s in c["pname"]]),
        int_column("price", c["price"], INT64),
        int_column("sname", codes(c["sname"]), CATEGORICAL),
        string_column("description", [None if s is None else s.encode() for s in c["description"]]),
        int_column("color", codes(c["color"]), CATEGORICAL),
        string_column("saddress", [None if s is None else s.encode() for s in c["saddress"]]),
    ]
    rel = Relation(cols, 5)
    pname, price, sname, desc, color, saddr = 1, 2, 3, 4, 5, 6
    preds = {
        "sname=": Pred(EQ, sname),
        "description~JD": Pred(JACCARD, desc, q=3, num=0, den=1),
    }
    rules = {
        "phi1": [Pred(EQ, color), Pred(EQ, price), Pred(EQ, sname), Pred(ED, pname, k=13)],
        "phi2": [Pred(EQ, sname), Pred(JACCARD, desc, q=3, num=1, den=5)],
        "phi3": [Pred(ED, saddr, k=10), Pred(JACCARD, desc, q=3, num=1, den=5)],
    }
    return g, rel, rules, preds


def test_table1_examples():
    g, rel, rules, preds = _table1()
    for e in g["expect"]:
        i, j = e["pair"]
        if "rule" in e:
            assert oracle.rule_witness(rel, rules[e["rule"]], i, j) == e["witness"], e["what"]
            assert oracle.rule_witness(rel, rules[e["rule"]], j, i) == e["witness"], e["what"]
        else:
            assert oracle.sat(rel, preds[e["pred"]], i, j) == e["sat"], e["what"]


def test_table1_missing_fails_every_predicate():
    g, rel, rules, preds = _table1()
    price, desc, saddr = 2, 4, 6
    # t2's price, t5's description, t4's saddress are missing
    for p, row in ((Pred(EQ, price), 1), (Pred(ABSDIFF, price, d=10 ** 6), 1),
                   (Pred(JACCARD, desc, q=2, num=0, den=1), 4), (Pred(ED, desc, k=1000), 4),
                   (Pred(EQ, desc), 4), (Pred(ED, saddr, k=1000), 3)):
        for other in range(5):
            assert not oracle.sat(rel, p, row, other)
            assert not oracle.sat(rel, p, other, row)


def test_table1_blocking_full_mode():
    g, rel, rules, preds = _table1()
    out = oracle.blocking(rel, [rules["phi1"], rules["phi2"], rules["phi3"]], mode="full")
    pairs = {(int(x >> 32), int(x & 0xFFFFFFFF)) for x in out}
    assert (0, 3) in pairs and (3, 4) in pairs
    with pytest.raises(ValueError):   # phi3 has no equality to block on
        oracle.blocking(rel, [rules["phi3"]], mode="blocked")


def _rand(seed, **kw):
    return workloads.random_small(seed, **kw)


def _unpack(a):
    return {(int(x >> 32), int(x & 0xFFFFFFFF)) for x in a}


@pytest.mark.parametrize("seed", range(6))
def test_blocked_equals_full(seed):
    rel, rules = _rand(seed, n=120)
    a = oracle.blocking(rel, rules, "blocked")
    b = oracle.blocking(rel, rules, "full", threads=4)
    assert np.array_equal(a, b)
    assert np.all(np.diff(a.astype(np.int64)) > 0)


@pytest.mark.parametrize("seed", range(4))
def test_symmetry_row_reversal(seed):
    rel, rules = _rand(100 + seed, n=150)
    n = rel.n_rows
    rev = rel.take(list(range(n - 1, -1, -1)))
    a = _unpack(oracle.blocking(rel, rules))
    b = _unpack(oracle.blocking(rev, rules))
    assert a == {(min(n - 1 - i, n - 1 - j), max(n - 1 - i, n - 1 - j)) for i, j in b}


@pytest.mark.parametrize("seed", range(4))
def test_order_independence(seed):
    rel, rules = _rand(200 + seed, n=150)
    base = oracle.blocking(rel, rules)
    r = np.random.default_rng(seed)
    for _ in range(3):
        perm_rules = [list(rules[x]) for x in r.permutation(len(rules))]
        for rule in perm_rules:
            r.shuffle(rule)
        assert np.array_equal(oracle.blocking(rel, perm_rules, "full"), base)


@pytest.mark.parametrize("seed", range(3))
def test_partition_independence(seed):
    # with one key attribute, the key's value groups are independent: the
    # union of per-shard results (shards = sets of key values) is the result
    rel, rules = _rand(300 + seed, n=200, n_keys=1)
    base = _unpack(oracle.blocking(rel, rules))
    key = rel.columns[3]
    shard_of = {}
    rows_by_shard = {0: [], 1: [], 2: []}
    for i in range(rel.n_rows):
        v = key.get(i) if key.is_valid(i) else None
        s = shard_of.setdefault(v, len(shard_of) % 3)
        rows_by_shard[s].append(i)
    union = set()
    for s, rows in rows_by_shard.items():
        sub = rel.take(rows)
        for i, j in _unpack(oracle.blocking(sub, rules)):
            a, b = rows[i], rows[j]
            union.add((min(a, b), max(a, b)))
    assert union == base


@pytest.mark.parametrize("seed", range(4))
def test_monotonicity(seed):
    rel, rules = _rand(400 + seed, n=150)
    base = _unpack(oracle.blocking(rel, rules))
    looser = []
    for rule in rules:
        nr = []
        for p in rule:
            if p.op == ED:
                p = Pred(ED, p.attr, k=p.k + 2)
            elif p.op == JACCARD:
                p = Pred(JACCARD, p.attr, q=p.q, num=max(0, p.num - 1), den=p.den)
            elif p.op == ABSDIFF:
                p = Pred(ABSDIFF, p.attr, d=p.d + 3)
            nr.append(p)
        looser.append(nr)
    assert base <= _unpack(oracle.blocking(rel, looser))


@pytest.mark.parametrize("seed", range(4))
def test_union_of_rule_sets(seed):
    rel, rules = _rand(500 + seed, n=150, n_rules=6)
    a = _unpack(oracle.blocking(rel, rules[:3]))
    b = _unpack(oracle.blocking(rel, rules[3:]))
    assert _unpack(oracle.blocking(rel, rules)) == a | b


def test_exact_duplicates_always_match():
    rel, rules = _rand(600, n=100, null_p=0.0)
    n = rel.n_rows
    rows = list(range(n)) + list(range(n))
    doubled = rel.take(rows)
    got = _unpack(oracle.blocking(doubled, rules))
    for i in range(n):
        assert (i, i + n) in got


def test_person_small_matches_are_mostly_duplicates():
    rel, rules = workloads.person_small()
    got = _unpack(oracle.blocking(rel, rules))
    truth = {(min(i, int(s)), max(i, int(s))) for i, s in enumerate(rel.dup_src) if s >= 0}
    assert len(got & truth) > 0.5 * len(truth)
    assert len(got - truth) < 0.2 * len(got)


# ----------------------------------------------------------- candidate count

def _group_pairs(cols_values):
    keys = list(zip(*cols_values))
    _, cnt = np.unique(np.array(keys), axis=0, return_counts=True)
    return int((cnt * (cnt - 1) // 2).sum())


def test_candidate_count_closed_form_one_key():
    rel, rules = workloads.person_small()
    z = rel.columns[rel.col("zip")].values
    assert oracle.candidate_count(rel, rules) == _group_pairs([z])


@pytest.mark.parametrize("seed", range(3))
def test_candidate_count_inclusion_exclusion_two_keys(seed):
    rel, _ = _rand(700 + seed, n=250, null_p=0.0)
    k0, k1 = 3, 4
    rules = [[Pred(EQ, k0)], [Pred(EQ, k1), Pred(ED, 0, k=1)]]
    a = rel.columns[k0].values
    b = rel.columns[k1].values
    expect = _group_pairs([a]) + _group_pairs([b]) - _group_pairs([a, b])
    assert oracle.candidate_count(rel, rules) == expect


# ------------------------------------------------------- |a - b| <= d (range)

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def _absdiff_sat(a, b, d):
    rel = Relation([int_column("v", [a, b], INT64)], 2)
    return oracle.sat(rel, Pred(ABSDIFF, 0, d=d), 0, 1)


# (a, b, d, expected), each expected value worked out by hand from the
# difference written beside it
_ABSDIFF_CASES = [
    (5, 3, 2, True),     # difference 2 = d
    (3, 5, 2, True),     # the same pair the other way round
    (5, 3, 1, False),    # difference 2 = d + 1
    (5, 3, 3, True),     # difference 2 = d - 1
    (7, 7, 0, True),     # d = 0: equal values
    (7, 8, 0, False),    # d = 0: difference 1
    (-4, 4, 8, True),    # across zero: difference 8 = d
    (-4, 4, 7, False),   # difference 8 = d + 1
    (I64_MAX, 0, I64_MAX, True),           # difference 2^63 - 1 = d
    (I64_MAX, 0, I64_MAX - 1, False),      # difference 2^63 - 1 = d + 1
    (0, I64_MIN, I64_MAX, False),          # difference 2^63 > every int64 d
    (I64_MAX, -1, I64_MAX, False),         # difference 2^63: wraps to INT64_MIN in 64 bits
    (I64_MAX, I64_MIN, I64_MAX, False),    # difference 2^64 - 1: wraps to -1 in 64 bits
    (I64_MIN, I64_MAX, 0, False),          # the same, the other way round
    (I64_MIN, I64_MIN + 1, 0, False),      # difference 1 at the bottom of the range
    (I64_MIN, I64_MIN + 1, 1, True),
    (I64_MAX - 2, I64_MAX, 2, True),       # difference 2 at the top of the range
    (I64_MAX - 2, I64_MAX, 1, False),
]


@pytest.mark.parametrize("a,b,d,want", _ABSDIFF_CASES)
def test_absdiff_hand_worked(a, b, d, want):
    assert _absdiff_sat(a, b, d) is want
    assert _absdiff_sat(b, a, d) is want


def test_absdiff_count_closed_form():
    """For a fixed a and d, exactly 2d + 1 integers b have |a - b| <= d (the
    window a - d .. a + d); a strict test would count 2d - 1, a one-sided
    one d + 1."""
    bs = list(range(-40, 41))
    rel = Relation([int_column("v", [0] + bs, INT64)], 1 + len(bs))
    for d in range(0, 12):
        got = sum(oracle.sat(rel, Pred(ABSDIFF, 0, d=d), 0, 1 + x) for x in range(len(bs)))
        assert got == 2 * d + 1, d

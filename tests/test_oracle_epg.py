"""Pins of the plan-generator arithmetic (Section 4.2) against the paper's
worked examples 5-8 and closed forms of the selectivity estimate (CPU)."""
import math

import numpy as np
import pytest

from oracle import epg

# Predicates of Example 2 (phi1, phi2, phi3), ids in first-appearance order.
COLOR, PRICE, SNAME, PNAME, DESC, SADDR = range(6)
PHI1 = [COLOR, PRICE, SNAME, PNAME]
PHI2 = [SNAME, DESC]
PHI3 = [SADDR, DESC]
RULES = [PHI1, PHI2, PHI3]

# Values stated by Examples 6 and 8: sp(color) = 1, sp(pname) = 0.4,
# cost(color) = 0.1, cost(pname) = 0.6, sp(sname) = 0.4, sp(desc) = 0.2,
# wp(phi1) = 0.048 (which, with the others, fixes sp(price) = 0.3).
# Values the examples leave free are chosen so that Example 7 (phi1's path
# starts with sname=, shared with phi2) and Example 5 (the root has two
# children, sname= explored first) hold: sp(saddr) = 0.3 and the costs below.
SP = [1.0, 0.3, 0.4, 0.4, 0.2, 0.3]
COST = [0.1, 0.2, 0.1, 0.6, 1.0, 0.6]


def test_example6_pname_before_color():
    ce = [epg.cost_effectiveness(s, c) for s, c in zip(SP, COST)]
    assert ce[COLOR] == 0.0
    assert math.isclose(ce[PNAME], (1 - 0.4) / 0.6)
    order = epg.order_predicates(SP, COST)
    assert order.index(PNAME) < order.index(COLOR)


def test_example8_witness_probability_and_edge_score():
    assert math.isclose(epg.witness_probability(PHI2, SP), 0.08)
    assert math.isclose(epg.witness_probability(PHI1, SP), 0.048)
    order = epg.order_predicates(SP, COST)
    root, paths = epg.build_tree(RULES, order)
    epg.score_edges(RULES, paths, SP)
    n1 = paths[0][0]
    assert n1 is paths[1][0] and n1.pred == SNAME          # shared edge (N0, N1)
    assert math.isclose(n1.score, max(0.048, 0.08))


def test_example7_tree_shape():
    order = epg.order_predicates(SP, COST)
    root, paths = epg.build_tree(RULES, order)
    # phi1 makes the path N0 -> N1 -> N2 -> N3 -> N4, phi2 re-uses N1 and adds N5
    assert [n.pred for n in paths[0]] == [SNAME, PRICE, PNAME, COLOR]
    assert paths[1][0] is paths[0][0]
    assert paths[1][1] is not paths[0][1] and paths[1][1].pred == DESC
    assert len(root.children) == 2          # sname= and phi3's first edge
    assert paths[0][-1].rules == [0] and paths[1][-1].rules == [1]


def test_example5_dfs_order():
    seq, root, paths = epg.sequential_path(RULES, SP, COST)
    assert [r for r, _ in seq] == [1, 0, 2]                 # phi2, phi1, phi3
    assert seq[0][1] == [SNAME, DESC]


def test_prefix_rule_visited_before_children():
    rules = [[0, 1], [0]]
    seq, _, _ = epg.sequential_path(rules, [0.5, 0.5], [0.5, 0.1])
    assert [r for r, _ in seq] == [1, 0]


def test_tree_has_one_leaf_per_rule_and_paths_cover_predicates():
    r = np.random.default_rng(3)
    for _ in range(50):
        n_p = int(r.integers(1, 9))
        rules = [list(r.choice(n_p, size=int(r.integers(1, n_p + 1)), replace=False)) for _ in range(int(r.integers(1, 7)))]
        sp = list(r.random(n_p))
        cost = list(r.random(n_p) + 0.01)
        seq, root, paths = epg.sequential_path(rules, sp, cost)
        assert sorted(x for x, _ in seq) == list(range(len(rules)))
        order = epg.order_predicates(sp, cost)
        rank = {p: i for i, p in enumerate(order)}
        for x, preds in seq:
            assert sorted(preds) == sorted(set(rules[x]))
            assert [rank[p] for p in preds] == sorted(rank[p] for p in preds)


# -------------------------------------------------------------- selectivity

def test_sp_all_in_one_bucket_is_one():
    b = np.zeros(epg.LSH_K, dtype=np.int64)
    b[17] = 500
    assert math.isclose(epg.sp_from_counts(b, 500), 1.0)
    assert math.isclose(epg.sp_from_counts_float(b, 500), 1.0)


def test_sp_perfectly_even_is_zero():
    b = np.full(epg.LSH_K, 3, dtype=np.int64)
    assert epg.sp_from_counts(b, 3 * epg.LSH_K) == 0.0
    assert epg.sp_from_counts_float(b, 3 * epg.LSH_K) < 1e-12


@pytest.mark.parametrize("seed", range(5))
def test_sp_integer_form_matches_paper_formula(seed):
    r = np.random.default_rng(seed)
    b = r.integers(0, 50, size=epg.LSH_K)
    n = int(b.sum())
    assert math.isclose(epg.sp_from_counts(b, n), epg.sp_from_counts_float(b, n), rel_tol=1e-9)


def test_mix64_and_fnv_published_vectors():
    # splitmix64 with state 0 yields 0xE220A8397B1DCDAF as its first output:
    # the output function applied to 0x9E3779B97F4A7C15
    assert epg.mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    # FNV-1a 64: offset basis for the empty input, and the "a" test vector
    assert epg.fnv1a64(b"") == 0xCBF29CE484222325
    assert epg.fnv1a64(b"a") == 0xAF63DC4C8601EC8C


def test_mix64_published_stream():
    # the first four outputs of splitmix64 from state 0: the output function
    # of s * 0x9E3779B97F4A7C15 for s = 1..4 (Steele, Lea and Flood 2014)
    g = 0x9E3779B97F4A7C15
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert [epg.mix64((s * g) & epg.MASK) for s in range(1, 5)] == want
    assert epg.mix64(0) == 0   # every step of the output function keeps 0 at 0


# ------------------------------------------------ LSH buckets (selectivity)
# The buckets only order the plan (they never change which pairs match), so
# sp itself stays unpinned; these pin the bucket functions the estimate and
# the device histograms are built from.

def _cols(values=None, strings=None):
    from gen import INT64, STRING, int_column, string_column
    if strings is not None:
        return string_column("s", strings)
    return int_column("v", values, INT64)


def test_gram_code_injective():
    """Distinct strings of up to 4 bytes get distinct codes: exhaustively
    over every string of at most 2 bytes, and up to 4 bytes over an alphabet
    holding the extreme byte values."""
    import itertools
    seen = {}
    for L in range(3):
        for t in itertools.product(range(256), repeat=L):
            s = bytes(t)
            c = epg.gram_code(s)
            assert c not in seen, (s, seen.get(c))
            seen[c] = s
    alpha = [0x00, 0x01, 0x61, 0x62, 0x7F, 0x80, 0xFE, 0xFF]
    seen = {}
    for L in range(5):
        for t in itertools.product(alpha, repeat=L):
            s = bytes(t)
            c = epg.gram_code(s)
            assert c not in seen, (s, seen.get(c))
            seen[c] = s


def test_gram_code_hand_values():
    assert epg.gram_code(b"") == 0
    assert epg.gram_code(b"a") == 0x1_00000061
    assert epg.gram_code(b"ab") == 0x2_00006162
    assert epg.gram_code(b"\x00") == 0x1_00000000        # not the empty string's code
    assert epg.gram_code(b"\x00\x00") == 0x2_00000000    # nor the one-byte zero's
    assert epg.gram_code(b"\xff\xff\xff\xff") == 0x4_FFFFFFFF


def test_equality_bucket_of_a_published_value():
    # the value whose splitmix64 output is published: 0xE220A8397B1DCDAF
    # mod 1024 = 0x1AF = 431 (the value as an int64 is negative)
    v = 0x9E3779B97F4A7C15 - (1 << 64)
    col = _cols(values=[v, 0])
    from gen import EQ, Pred
    assert epg.lsh_bucket(col, Pred(EQ, 0), 0) == 431
    assert epg.lsh_bucket(col, Pred(EQ, 0), 1) == 0     # the output function maps 0 to 0


def test_range_buckets_group_windows_of_d_plus_one():
    from gen import ABSDIFF, Pred
    for d in (0, 1, 4, 9):
        vals = list(range(-2 * (d + 1), 3 * (d + 1)))
        col = _cols(values=vals)
        b = [epg.lsh_bucket(col, Pred(ABSDIFF, 0, d=d), i) for i in range(len(vals))]
        for i, v in enumerate(vals):
            if 0 <= v <= d:
                assert b[i] == 0, (d, v)    # floor(v / (d + 1)) = 0, and 0 maps to bucket 0
            # v and v + d + 1 are a window apart: same offset in the next window
            same = [b[x] for x, w in enumerate(vals) if w // (d + 1) == v // (d + 1)]
            assert len(set(same)) == 1 and len(same) == d + 1


def test_minhash_equal_gram_sets_equal_buckets():
    from gen import ED, JACCARD, Pred
    # pairs of different strings with the same gram set
    same_sets = [(b"abab", b"baba", 2), (b"aaaa", b"aa", 2), (b"abcabc", b"bcabca", 3), (b"xy", b"xy", 3)]
    for a, b, q in same_sets:
        assert epg.qgram_set(a, q) == epg.qgram_set(b, q)
        col = _cols(strings=[a, b])
        p = Pred(JACCARD, 0, q=q, num=1, den=2)
        assert epg.lsh_bucket(col, p, 0) == epg.lsh_bucket(col, p, 1)
        if q == 2:
            pe = Pred(ED, 0, k=1)
            assert epg.lsh_bucket(col, pe, 0) == epg.lsh_bucket(col, pe, 1)


def test_minhash_is_the_least_gram_hash():
    for s, q in ((b"kitten", 2), (b"sitting", 3), (b"ab", 3), (b"mississippi", 2)):
        hs = [epg.mix64(epg.gram_code(g)) for g in epg.qgram_set(s, q)]
        assert epg.minhash(s, q) == min(hs)
    assert epg.minhash(b"", 2) == 0          # no gram: the reading's value
    # a string shorter than q is its own single gram
    assert epg.minhash(b"ab", 3) == epg.mix64(0x2_00006162)

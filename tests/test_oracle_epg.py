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

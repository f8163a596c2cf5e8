"""The quality report (precision, recall, F1, CSSR as the experimental
section defines them) and the ground truth drawn from the generator's
duplicate links, pinned on hand-counted cases and against a set-based
brute force.  CPU only."""
import itertools

import numpy as np
import pytest

from gen import Relation, entity_ids, int_column, true_pairs, workloads
from paper_2410_04349_amd.quality import quality


def pack(pairs):
    return np.array(sorted((min(a, b) << 32) | max(a, b) for a, b in pairs), dtype=np.uint64)


def test_hand_counted_case():
    # truth: {0,1,2} one entity (3 pairs), {3,4} another (1 pair)
    truth = pack([(0, 1), (0, 2), (1, 2), (3, 4)])
    got = pack([(0, 1), (1, 2), (2, 3)])          # 2 right, 1 wrong
    q = quality(got, truth, n_rows=6)
    assert q["true_identified"] == 2 and q["identified"] == 3 and q["true_pairs"] == 4
    assert q["precision"] == pytest.approx(2 / 3)
    assert q["recall"] == pytest.approx(1 / 2)
    assert q["f1"] == pytest.approx(2 * (2 / 3) * (1 / 2) / (2 / 3 + 1 / 2))
    assert q["cssr"] == pytest.approx(3 / 36)


def test_degenerate_cases():
    truth = pack([(0, 1)])
    assert quality(pack([]), truth, 4)["recall"] == 0.0 and quality(pack([]), truth, 4)["f1"] == 0.0
    q = quality(truth, truth, 4)
    assert q["precision"] == q["recall"] == q["f1"] == 1.0
    # order and repeats of the input do not matter
    assert quality(np.r_[truth, truth][::-1], truth, 4)["identified"] == 1


def test_true_pairs_from_duplicate_links():
    col = int_column("k", [0, 1, 2, 3, 4, 5])
    # rows 3 and 4 duplicate row 0, row 5 duplicates row 3 (a chain to 0)
    rel = Relation([col], 6, np.array([-1, -1, -1, 0, 0, 3]))
    assert entity_ids(rel).tolist() == [0, 1, 2, 0, 0, 0]
    want = pack(itertools.combinations([0, 3, 4, 5], 2))
    assert np.array_equal(true_pairs(rel), want)


def test_quality_matches_set_brute_force():
    rel, _ = workloads.person_small()
    truth = true_pairs(rel)
    ent = entity_ids(rel)
    groups = {}
    for i, e in enumerate(ent.tolist()):
        groups.setdefault(e, []).append(i)
    brute = {(a, b) for g in groups.values() for a, b in itertools.combinations(sorted(g), 2)}
    assert set((int(x) >> 32, int(x) & 0xFFFFFFFF) for x in truth) == brute
    r = np.random.default_rng(3)
    picked = [p for p in brute if r.random() < 0.7]
    noise = {(int(a), int(b)) for a, b in r.integers(0, rel.n_rows, size=(200, 2)) if a < b} - brute
    got = pack(picked + list(noise))
    q = quality(got, truth, rel.n_rows)
    assert q["true_identified"] == len(picked)
    assert q["precision"] == pytest.approx(len(picked) / (len(picked) + len(noise)))
    assert q["recall"] == pytest.approx(len(picked) / len(brute))

"""Properties of the seeded generator (CPU): determinism, the capped-Zipf
block cap and the key-correlated string columns."""
import numpy as np

from gen import workloads


def test_learned_recipe_deterministic_and_capped():
    a, rules_a = workloads.learned_10m(n=20_000)
    b, rules_b = workloads.learned_10m(n=20_000)
    assert rules_a == rules_b and len(rules_a) == 20
    for ca, cb in zip(a.columns, b.columns):
        if ca.values is not None:
            assert np.array_equal(ca.values, cb.values)
        else:
            assert np.array_equal(ca.offsets, cb.offsets) and np.array_equal(ca.data, cb.data)
    # base tuples per key code never exceed the cap (duplicates may add more)
    cap = max(8, int(round(5000 * min(1.0, 20_000 / 10_000_000 * 20))))
    base = a.dup_src < 0
    for key in (4, 5):
        _, cnt = np.unique(a.columns[key].values[base], return_counts=True)
        assert cnt.max() <= cap


def _strings(col):
    return [bytes(col.data[col.offsets[i]:col.offsets[i + 1]]) for i in range(len(col.offsets) - 1)]


def test_keyed_column_pinned_blocks():
    rel, _ = workloads.learned_10m(n=20_000)
    base = np.flatnonzero(rel.dup_src < 0)
    for key, col in ((4, 6), (5, 7)):
        codes = rel.columns[key].values
        s = _strings(rel.columns[col])
        groups = {}
        for r in base:
            groups.setdefault(int(codes[r]), []).append(s[r])
        big = [g for g in groups.values() if len(g) >= 8]
        pinned = [g for g in big if len(set(g)) == 1]
        free = [g for g in big if len(set(g)) == len(g)]
        # about 30% of the codes pin their string; the rest draw freely
        assert len(pinned) + len(free) == len(big)
        assert 0.15 < len(pinned) / len(big) < 0.45, (len(pinned), len(big))

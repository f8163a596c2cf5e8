"""Named synthetic workloads (relations + rule sets).

These stand in for the paper's real datasets (Table 2), which are not
available.  Each workload is seeded; the recipe of each is stated here and
restated in the design notes.

  person_small   2,000 person tuples (1,600 base + 400 duplicates made by 1-2
                 char edits on name/address); name a-z len 5-20, address
                 a-z0-9-space len 20-40, zip uniform over 200 random 5-digit
                 codes, age 18-90; one rule
                 zip= AND ED(name)<=2 AND J3(address)>=3/5.
  plain_1m       1,000,000 tuples (850k base + 150k duplicates, 1-3 char edits
                 over s1..s3, each int shifted by U{-2..2} with p=0.3);
                 s1,s2,s3 a-z-space len 5-40; key capped Zipf s=1.1 over 50k
                 values, cap 5,000 base tuples per code; i1 U[0,99];
                 i2 U[1900,2024]; five rules of 3-4 predicates.
  learned_10m    10,000,000 tuples (9M base + 1M duplicates, 1-3 char edits,
                 ints shifted by U{-2..2} with p=0.3); s1..s4 a-z-space len
                 5-60; k1, k2 capped Zipf s=1.2 over 500k values, cap 5,000;
                 s5 (following k1) and s6 (following k2) a-z-space len 5-60,
                 pinned to one string per key code with p=0.3; i1 U[0,99],
                 i2 U[1900,2024]; 20 seeded rules, 10 per key, each the key
                 equality, one predicate on s1..s4 and 1-3 more from the
                 plain menu (ED<=1..3, J3>=1/2..4/5, |diff|<=2).
  long_titles_5m 5,000,000 product titles (4.5M base + 0.5M duplicates with
                 1-8 char edits); title = pseudo-words (30k words of 2-10
                 a-z letters, Zipf s=1.0 word frequencies) cut to a length
                 U[20, 200]; brand capped Zipf s=1.3 over 100k values with
                 cap 18, the smallest cap giving 50M +- 10% candidate pairs
                 (46,306,524 at 5M); one rule
                 brand= AND J2(title)>=7/10 AND ED(title)<=8.
  batched_64     64 independent relations with sizes log-uniform in
                 [10k, 2M] tuples (each the plain recipe: 15% duplicates,
                 key capped Zipf s=1.1 with 50 values per 1,000 tuples, cap
                 5,000), each with its own 1-10 rules: the key equality, one
                 string predicate and 0-2 more from the plain menu.
  random_small   adversarial small relations for parity (lengths 0, q-1,
                 63/64/65, 127/128/129, 200; nulls; tiny alphabets; several
                 keys; rule sets with the key equality anywhere in a rule).
"""
from __future__ import annotations

import numpy as np

from . import (ABSDIFF, CATEGORICAL, ED, EQ, EQ_CONST, INT64, JACCARD, STRING, AttrSpec,
               Column, Pred, Relation, generate, pack_bits)

SEED_BASE = 0x48420000


def person_small(seed: int = SEED_BASE + 1):
    attrs = [
        AttrSpec("name", "string", alphabet=0, min_len=5, max_len=20, editable=True),
        AttrSpec("address", "string", alphabet=1, min_len=20, max_len=40, editable=True),
        AttrSpec("zip", "codes", n_values=200, lo=10000, hi=99999, editable=False),
        AttrSpec("age", "int", lo=18, hi=90),
    ]
    rel = generate(seed, 1600, 400, attrs, edit_min=1, edit_max=2)
    name, address, zip_ = rel.col("name"), rel.col("address"), rel.col("zip")
    rules = [[Pred(EQ, zip_), Pred(ED, name, k=2), Pred(JACCARD, address, q=3, num=3, den=5)]]
    return rel, rules


def plain_1m_attrs(n_values: int = 50_000, cap: int = 5000):
    return [
        AttrSpec("s1", "string", alphabet=2, min_len=5, max_len=40),
        AttrSpec("s2", "string", alphabet=2, min_len=5, max_len=40),
        AttrSpec("s3", "string", alphabet=2, min_len=5, max_len=40),
        AttrSpec("key", "zipf", zipf_s=1.1, n_values=n_values, cap=cap),
        AttrSpec("i1", "int", lo=0, hi=99, int_p=0.3, int_d=2),
        AttrSpec("i2", "int", lo=1900, hi=2024, int_p=0.3, int_d=2),
    ]


def plain_1m_rules():
    s1, s2, s3, key, i1, i2 = range(6)
    return [
        [Pred(EQ, key), Pred(ED, s1, k=2), Pred(JACCARD, s2, q=3, num=3, den=5)],
        [Pred(EQ, key), Pred(ABSDIFF, i1, d=2), Pred(ED, s2, k=1), Pred(JACCARD, s3, q=3, num=1, den=2)],
        [Pred(EQ, key), Pred(JACCARD, s1, q=3, num=7, den=10), Pred(ED, s3, k=3)],
        [Pred(EQ, key), Pred(ABSDIFF, i2, d=2), Pred(ED, s1, k=3), Pred(JACCARD, s3, q=3, num=4, den=5)],
        [Pred(EQ, key), Pred(JACCARD, s2, q=3, num=1, den=2), Pred(ABSDIFF, i1, d=2), Pred(ED, s3, k=2)],
    ]


def plain_1m_ordered_rules():
    """plain_1m's rules plus one that tells t from s: t.i1 = 7 and
    ED(s1) <= 3.  The rule set is ordered (each symmetric match is listed
    in both orders)."""
    s1, s2, s3, key, i1, i2 = range(6)
    return plain_1m_rules() + [[Pred(EQ, key), Pred(EQ_CONST, i1, side=0, c=7), Pred(ED, s1, k=3)]]


def plain_1m(seed: int = SEED_BASE + 2, n: int = 1_000_000):
    """The 1M-tuple plain workload; `n` scales it down (same recipe, 15%
    duplicates, Zipf values and cap scaled with n) for parity tests."""
    n_dup = (n * 15) // 100
    scale = n / 1_000_000
    n_values = max(50, int(round(50_000 * scale)))
    cap = max(8, int(round(5000 * min(1.0, scale * 20))))
    rel = generate(seed, n - n_dup, n_dup, plain_1m_attrs(n_values, cap), edit_min=1, edit_max=3)
    return rel, plain_1m_rules()


# ------------------------------------------------------------ learned 10M

def learned_10m_attrs(n_values: int = 500_000, cap: int = 5000):
    free = [AttrSpec(f"s{x}", "string", alphabet=2, min_len=5, max_len=60) for x in range(1, 5)]
    return free + [
        AttrSpec("k1", "zipf", zipf_s=1.2, n_values=n_values, cap=cap),
        AttrSpec("k2", "zipf", zipf_s=1.2, n_values=n_values, cap=cap),
        AttrSpec("s5", "keyed", alphabet=2, min_len=5, max_len=60, dep=4, dep_p=0.3),
        AttrSpec("s6", "keyed", alphabet=2, min_len=5, max_len=60, dep=5, dep_p=0.3),
        AttrSpec("i1", "int", lo=0, hi=99, int_p=0.3, int_d=2),
        AttrSpec("i2", "int", lo=1900, hi=2024, int_p=0.3, int_d=2),
    ]


def learned_10m_rules(seed: int = SEED_BASE + 3):
    """20 rules, 10 per key: key equality, one predicate on a free string
    (s1..s4) and 1-3 more drawn from the plain menu over every non-key
    attribute (no attribute twice in a rule)."""
    r = np.random.default_rng(seed)
    free, keyed, ints = [0, 1, 2, 3], [6, 7], [8, 9]
    jac = [(1, 2), (3, 5), (7, 10), (4, 5)]

    def string_pred(a):
        if r.random() < 0.5:
            return Pred(ED, a, k=int(r.integers(1, 4)))
        num, den = jac[int(r.integers(0, len(jac)))]
        return Pred(JACCARD, a, q=3, num=num, den=den)

    rules = []
    for key in (4, 5):
        for _ in range(10):
            anchor = free[int(r.integers(0, len(free)))]
            rule = [Pred(EQ, key), string_pred(anchor)]
            others = [a for a in free + keyed + ints if a != anchor]
            for a in r.choice(others, size=int(r.integers(1, 4)), replace=False):
                a = int(a)
                rule.append(Pred(ABSDIFF, a, d=2) if a in ints else string_pred(a))
            rules.append(rule)
    return rules


def learned_10m(seed: int = SEED_BASE + 4, n: int = 10_000_000):
    """The 10M-tuple two-key workload; `n` scales it down (same recipe, key
    cardinality and cap scaled with n) for parity tests."""
    n_dup = n // 10
    scale = n / 10_000_000
    n_values = max(50, int(round(500_000 * scale)))
    cap = max(8, int(round(5000 * min(1.0, scale * 20))))
    rel = generate(seed, n - n_dup, n_dup, learned_10m_attrs(n_values, cap), edit_min=1, edit_max=3)
    return rel, learned_10m_rules()


# ------------------------------------------------------------ batched 64

def batched_rules(r: np.random.Generator, n_rules: int):
    s_attrs, key, ints = [0, 1, 2], 3, [4, 5]
    jac = [(1, 2), (3, 5), (7, 10), (4, 5)]

    def string_pred(a):
        if r.random() < 0.5:
            return Pred(ED, a, k=int(r.integers(1, 4)))
        num, den = jac[int(r.integers(0, len(jac)))]
        return Pred(JACCARD, a, q=3, num=num, den=den)

    rules = []
    for _ in range(n_rules):
        anchor = s_attrs[int(r.integers(0, 3))]
        rule = [Pred(EQ, key), string_pred(anchor)]
        others = [a for a in s_attrs + ints if a != anchor]
        for a in r.choice(others, size=int(r.integers(0, 3)), replace=False):
            a = int(a)
            rule.append(Pred(ABSDIFF, a, d=2) if a in ints else string_pred(a))
        rules.append(rule)
    return rules


def batched_64(seed: int = SEED_BASE + 6, n_jobs: int = 64, lo: int = 10_000, hi: int = 2_000_000,
               scale: float = 1.0, cap: int = 5000):
    """[(relation, rules)] of the batched workload; `scale` multiplies every
    relation size and `cap` bounds the blocks (smaller for parity tests)."""
    r = np.random.default_rng(seed)
    sizes = np.exp(r.uniform(np.log(lo), np.log(hi), size=n_jobs))
    out = []
    for k, size in enumerate(sizes):
        n = max(40, int(round(size * scale)))
        n_dup = (n * 15) // 100
        n_values = max(8, int(round(n * 0.05)))
        rel = generate(seed * 1000 + k, n - n_dup, n_dup, plain_1m_attrs(n_values, cap), edit_min=1, edit_max=3)
        out.append((rel, batched_rules(r, int(r.integers(1, 11)))))
    return out


# ------------------------------------------------------------ long titles

def long_titles_5m(seed: int = SEED_BASE + 5, n: int = 5_000_000):
    """Long strings and skewed keys; `n` scales it down (brand cardinality
    scaled with n, the cap of 18 tuples per code kept)."""
    n_dup = n // 10
    n_values = max(50, int(round(100_000 * n / 5_000_000)))
    attrs = [
        AttrSpec("brand", "zipf", zipf_s=1.3, n_values=n_values, cap=18),
        AttrSpec("title", "words", min_len=20, max_len=200, zipf_s=1.0, n_values=30_000),
    ]
    rel = generate(seed, n - n_dup, n_dup, attrs, edit_min=1, edit_max=8)
    rules = [[Pred(EQ, 0), Pred(JACCARD, 1, q=2, num=7, den=10), Pred(ED, 1, k=8)]]
    return rel, rules


# ------------------------------------------------------------ adversarial

_LEN_MENU = [0, 1, 2, 3, 5, 31, 32, 33, 63, 64, 65, 127, 128, 129, 200]


def _sm64(x):
    x = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return x, z ^ (z >> 31)


class _Rng:
    """splitmix64 stream (Steele, Lea and Flood 2014); small and portable."""

    def __init__(self, seed: int):
        self.x = seed & 0xFFFFFFFFFFFFFFFF

    def next(self) -> int:
        self.x, z = _sm64(self.x)
        return z

    def below(self, n: int) -> int:
        return self.next() % n if n > 1 else 0

    def unit(self) -> float:
        return (self.next() >> 11) / float(1 << 53)


def random_small(seed: int, n: int = 300, n_str: int = 3, n_keys: int = 2, n_ints: int = 1,
                 alphabet: bytes = b"ab", null_p: float = 0.05, n_key_values: int = 8,
                 n_rules: int = 4, long_strings: bool = True, dup_p: float = 0.3):
    """A small adversarial relation and rule set.

    Strings draw their length from a menu of boundary lengths (0, 1, 2, q-1,
    31/32/33, 63/64/65, 127/128/129, 200) when `long_strings`, else U[0,12],
    over a tiny alphabet so that similarity predicates pass often.  About
    `dup_p` of the rows copy an earlier row and apply one or two edits, so
    matches occur.  Each attribute value is missing with probability `null_p`.
    Rules have 1-4 predicates and each carries an equality on some key, at a
    random position in the rule.
    """
    r = _Rng(seed)
    strs = [[None] * n for _ in range(n_str)]
    keys = [[None] * n for _ in range(n_keys)]
    ints = [[None] * n for _ in range(n_ints)]
    for i in range(n):
        src = r.below(i) if (i > 0 and r.unit() < dup_p) else -1
        for a in range(n_str):
            if src >= 0 and strs[a][src] is not None:
                s = bytearray(strs[a][src])
                for _ in range(1 + r.below(2)):
                    t = r.below(3)
                    if t == 0 and len(s):
                        s[r.below(len(s))] = alphabet[r.below(len(alphabet))]
                    elif t == 1:
                        s.insert(r.below(len(s) + 1), alphabet[r.below(len(alphabet))])
                    elif len(s):
                        del s[r.below(len(s))]
                strs[a][i] = bytes(s)
            else:
                L = _LEN_MENU[r.below(len(_LEN_MENU))] if long_strings else r.below(13)
                strs[a][i] = bytes(alphabet[r.below(len(alphabet))] for _ in range(L))
        for a in range(n_keys):
            if src >= 0 and r.unit() < 0.9:
                keys[a][i] = keys[a][src]
            else:
                keys[a][i] = r.below(n_key_values) - (n_key_values // 2)
        for a in range(n_ints):
            if src >= 0 and ints[a][src] is not None:
                ints[a][i] = ints[a][src] + r.below(5) - 2
            else:
                ints[a][i] = r.below(40) - 20 if r.unit() < 0.9 else (r.next() >> 1) * (1 if r.unit() < 0.5 else -1)
    cols = []
    for a in range(n_str):
        vals = [None if r.unit() < null_p else v for v in strs[a]]
        from . import string_column
        cols.append(string_column(f"s{a}", vals))
    from . import int_column
    for a in range(n_keys):
        vals = [None if r.unit() < null_p else v for v in keys[a]]
        cols.append(int_column(f"k{a}", vals, CATEGORICAL if a % 2 == 0 else INT64))
    for a in range(n_ints):
        vals = [None if r.unit() < null_p else v for v in ints[a]]
        cols.append(int_column(f"i{a}", vals, INT64))
    rel = Relation(cols, n, None)

    str_ids = list(range(n_str))
    key_ids = list(range(n_str, n_str + n_keys))
    int_ids = list(range(n_str + n_keys, n_str + n_keys + n_ints))
    rules = []
    for _ in range(n_rules):
        preds = []
        for _ in range(r.below(4)):
            kind = (0, 0, 1, 1, 2, 3, 4)[r.below(7)]
            if kind == 0 and str_ids:
                preds.append(Pred(ED, str_ids[r.below(len(str_ids))], k=r.below(6)))
            elif kind == 1 and str_ids:
                den = 1 + r.below(10)
                preds.append(Pred(JACCARD, str_ids[r.below(len(str_ids))], q=1 + r.below(4),
                                  num=r.below(den + 1), den=den))
            elif kind == 2 and int_ids:
                preds.append(Pred(ABSDIFF, int_ids[r.below(len(int_ids))], d=r.below(4)))
            elif kind == 3:
                preds.append(Pred(EQ, (str_ids + int_ids)[r.below(len(str_ids + int_ids))]))
            else:
                preds.append(Pred(EQ, key_ids[r.below(len(key_ids))]))
        preds.insert(r.below(len(preds) + 1), Pred(EQ, key_ids[r.below(len(key_ids))]))
        rules.append(preds)
    return rel, rules

"""Per-pair cost network N -- oracle side, TEST INFRASTRUCTURE ONLY.

Follows Section 4.2 of the paper ("Evaluation cost", "Shallow NNs",
"Estimated cost"): the cost of a predicate p on D is the sum over tuple
pairs of D x D of the time T_p(t1, t2) its check takes; a small network N
estimates T_p from p and the two tuples' A-values, and the estimated cost is
norm(sum of N(p, t1, t2)), over a sample of the pairs in practice.

Readings where the paper is silent (also in the design notes):
  * the sample: pair s of a seed is i = h(seed + 2s) mod n,
    j = h(seed + 2s + 1) mod n, j replaced by (i + 1) mod n when equal to i
    (h = the splitmix64 output function); every predicate is estimated on
    the same sampled pairs;
  * the encoding of (p, t1.A, t2.A) is the 16 numbers of `pair_features`
    (predicate kind, presence, lengths, q-gram counts, thresholds), all of
    them integers scaled by powers of two or one rounded fraction, so that
    both sides compute them exactly;
  * N is the library's 16 -> 64 -> 64 -> 2 network; its second output y is
    log2(1 + clock cycles) / 16 of the check, so an estimate is
    2^(16 * clamp(y, 0, 4)) - 1 cycles;
  * norm() divides by the largest predicate's sum, with every cost kept at
    or above 2^-20 of it so that each lies in (0, 1]; when every sum is zero
    (or n < 2: no pairs) every cost is 1.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import epg, mlp

N_FEATURES = 16
KINDS = ("value_eq", "absdiff", "string_eq", "edit_distance", "jaccard")
COST_FLOOR = 2.0 ** -20
Y_CLAMP = 4.0


def sample_pair(seed: int, s: int, n: int) -> Tuple[int, int]:
    """Sampled pair s of D x D (n >= 2 tuples): two distinct row indexes."""
    i = epg.mix64(seed + 2 * s) % n
    j = epg.mix64(seed + 2 * s + 1) % n
    if j == i:
        j = (i + 1) % n
    return i, j


def kind(rel, pred) -> int:
    """Index in KINDS of a predicate comparing one attribute of both tuples;
    other predicate forms are outside this estimate (ValueError)."""
    col = rel.columns[pred.attr]
    if pred.op == "eq" or (pred.op == "eq_cross" and pred.attr_b == pred.attr):
        return 2 if col.type == "string" else 0
    if pred.op == "absdiff":
        return 1
    if pred.op == "ed" or (pred.op == "ed_cross" and pred.attr_b == pred.attr):
        return 3
    if pred.op == "jaccard" or (pred.op == "jaccard_cross" and pred.attr_b == pred.attr):
        return 4
    raise ValueError(f"no per-pair cost for {pred.op} across attributes")


def gram_count(s: bytes, q: int) -> int:
    """|G_q(s)|: distinct length-q windows; 1 for a non-empty string shorter
    than q; 0 for the empty string."""
    return len(epg.qgram_set(s, q))


def pair_features(rel, pred, i: int, j: int) -> np.ndarray:
    """The 16 inputs of N for predicate `pred` on tuples (i, j):
      0-4   one-hot predicate kind (value equality, |a-b| <= d, string
            equality, edit distance, q-gram Jaccard)
      5, 6  t1.A present, t2.A present
      7, 8  byte lengths L1 / 64, L2 / 64 (strings; 0 when missing)
      9     string equality: [L1 == L2] with both present;
            edit distance: pattern words W(L1) / 4, W(L) = 0 for L <= 32
            else ceil(L / 64); Jaccard: q-gram count C1 / 64
      10    edit distance: k / 16; Jaccard: C2 / 64
      11    Jaccard: 1 if either value is shorter than q (and not empty)
      12    Jaccard: num / den rounded to fp32
      13    min(L1, L2) / 64
      14    |L1 - L2| / 64
      15    1
    Counts and lengths of a missing value are 0."""
    f = np.zeros(N_FEATURES, dtype=np.float32)
    col = rel.columns[pred.attr]
    kd = kind(rel, pred)
    f[kd] = 1.0
    ok1, ok2 = col.is_valid(i), col.is_valid(j)
    f[5], f[6] = float(ok1), float(ok2)
    f[15] = 1.0
    if col.type != "string":
        return f
    a = col.get(i) if ok1 else b""
    b = col.get(j) if ok2 else b""
    l1, l2 = len(a), len(b)
    f[7], f[8] = l1 / 64.0, l2 / 64.0
    f[13] = min(l1, l2) / 64.0
    f[14] = abs(l1 - l2) / 64.0
    if kd == 2:
        f[9] = 1.0 if (ok1 and ok2 and l1 == l2) else 0.0
    elif kd == 3:
        words = 0 if l1 <= 32 else (l1 + 63) // 64
        f[9] = words / 4.0
        f[10] = pred.k / 16.0
    elif kd == 4:
        f[9] = gram_count(a, pred.q) / 64.0
        f[10] = gram_count(b, pred.q) / 64.0
        f[11] = 1.0 if (0 < l1 < pred.q) or (0 < l2 < pred.q) else 0.0
        f[12] = np.float32(pred.num / pred.den)
    return f


def sample_features(rel, preds: Sequence, samples: int, seed: int) -> np.ndarray:
    """Features of every predicate (outer) on every sampled pair (inner):
    [len(preds) * samples, 16]."""
    pairs = [sample_pair(seed, s, rel.n_rows) for s in range(samples)]
    return np.stack([pair_features(rel, p, i, j) for p in preds for (i, j) in pairs])


def bf16_forward(params, x) -> np.ndarray:
    """N's outputs with the library's arithmetic: every product's operands
    rounded to bf16 (hidden activations included), sums in fp64."""
    r = mlp.bf16_round
    z1 = r(x) @ r(params["W1"]) + params["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = r(h1) @ r(params["W2"]) + params["b2"]
    h2 = np.maximum(z2, 0.0)
    return r(h2) @ r(params["W3"]) + params["b3"]


def pair_cycles(y) -> np.ndarray:
    """Estimated cycles of each row from N's second output."""
    t = np.clip(np.asarray(y, dtype=np.float64)[:, 1], 0.0, Y_CLAMP)
    return np.exp2(16.0 * t) - 1.0


def estimated_costs(y, n_preds: int, samples: int) -> List[float]:
    """norm(sum over the sample of N's estimate), per predicate."""
    if n_preds == 0:
        return []
    if samples == 0:
        return [1.0] * n_preds
    sums = pair_cycles(y).reshape(n_preds, samples).sum(axis=1)
    top = float(sums.max())
    if not top > 0.0:
        return [1.0] * n_preds
    return [max(float(v), top * COST_FLOOR) / top for v in sums]

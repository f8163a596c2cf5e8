"""Execution-plan generator (EPG) arithmetic -- oracle side, TEST INFRASTRUCTURE ONLY.

Follows Section 4.2 of the paper ("Execution plan generation"):

  * selectivity  sp(p, D) = norm( sqrt( (1/k) * sum_i (b_i - |D|/k)^2 ) ),
    b_i = number of tuples whose A-value an LSH function puts in bucket i
    ("Effectiveness");
  * cost-effectiveness (1 - sp) / cost_hat, predicates ordered by it,
    descending ("Ordering scheme");
  * execution tree: each rule's predicates, sorted by that order, are
    inserted from the root, re-using an existing child edge with the same
    predicate ("Constructing an execution tree");
  * witness probability wp(phi) = product of sp over the rule's predicates;
    edge score = max wp over the rules whose root-to-leaf path contains the
    edge ("Edge score");
  * evaluation order: DFS from the root taking children by decreasing score
    ("Evaluating an execution plan"), flattened into the sequential execution
    path of Section 5.1 (rules in leaf-visit order, each with its predicates
    in root-to-leaf order).

Readings where the paper is silent (also in the design notes):
  * ties in cost-effectiveness keep the predicates' first-appearance order;
    ties in edge score keep the children's creation order;
  * a rule whose predicate set ends at an inner node (its predicates are a
    prefix of another rule's path) is visited on arrival at that node, before
    the node's children: reaching the node already makes it a witness;
    several rules ending at one node are visited in input order;
  * norm() for sp divides by the value reached when all tuples share one
    bucket, (|D|/k) * sqrt(k - 1), so sp lies in [0, 1] and equals 1 iff every
    tuple hashes to one bucket; with integer bucket counts this is
    sp = sqrt((k * sum b_i^2 - n^2) / (n^2 * (k - 1))); sp = 0 when n = 0;
  * the LSH functions (the paper names none) are: equality -> a hash of the
    value; |a-b| <= d -> a hash of floor(v / (d + 1)); edit distance -> one
    MinHash over the 2-gram set; Jaccard -> one MinHash over its own q-gram
    set; bucket = hash mod k, k = 1024; missing values are skipped.
    The hash is the splitmix64 output function (Steele, Lea and Flood 2014)
    and strings are first folded with FNV-1a 64 (Fowler, Noll and Vo).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

MASK = (1 << 64) - 1
LSH_K = 1024


# ---------------------------------------------------------------- selectivity

def mix64(x: int) -> int:
    z = x & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def fnv1a64(b: bytes) -> int:
    h = 0xCBF29CE484222325
    for c in b:
        h ^= c
        h = (h * 0x100000001B3) & MASK
    return h


def gram_code(g: bytes) -> int:
    """Code of a gram (or of a whole string shorter than q): its length in
    bits 32.. and its bytes big-endian below."""
    v = 0
    for c in g:
        v = (v << 8) | c
    return (len(g) << 32) | v


def qgram_set(s: bytes, q: int):
    if len(s) == 0:
        return set()
    if len(s) < q:
        return {s}
    return {s[x:x + q] for x in range(len(s) - q + 1)}


def minhash(s: bytes, q: int) -> int:
    g = qgram_set(s, q)
    if not g:
        return 0
    return min(mix64(gram_code(x)) for x in g)


def lsh_bucket(col, pred, i: int, k: int = LSH_K) -> int:
    if pred.op == "eq":
        if col.type == "string":
            return mix64(fnv1a64(col.get(i))) % k
        return mix64(col.get(i) & MASK) % k
    if pred.op == "absdiff":
        return mix64((col.get(i) // (pred.d + 1)) & MASK) % k
    if pred.op == "ed":
        return minhash(col.get(i), 2) % k
    if pred.op == "jaccard":
        return minhash(col.get(i), pred.q) % k
    raise ValueError(pred.op)


def bucket_counts(rel, pred, k: int = LSH_K) -> Tuple[np.ndarray, int]:
    col = rel.columns[pred.attr]
    b = np.zeros(k, dtype=np.int64)
    n = 0
    for i in range(rel.n_rows):
        if not col.is_valid(i):
            continue
        b[lsh_bucket(col, pred, i, k)] += 1
        n += 1
    return b, n


def sp_from_counts(b: Sequence[int], n: int, k: int = LSH_K) -> float:
    """norm(std-dev of bucket counts), evaluated from the integer counts."""
    if n == 0:
        return 0.0
    s2 = sum(int(x) * int(x) for x in b)
    num = k * s2 - n * n
    den = n * n * (k - 1)
    return math.sqrt(num / den)


def sp_from_counts_float(b: Sequence[int], n: int, k: int = LSH_K) -> float:
    """The same quantity, written as in the paper: sqrt((1/k) sum (b_i - n/k)^2)
    divided by its all-in-one-bucket value (n/k) sqrt(k-1)."""
    if n == 0:
        return 0.0
    sigma = math.sqrt(sum((float(x) - n / k) ** 2 for x in b) / k)
    return sigma / ((n / k) * math.sqrt(k - 1))


# ---------------------------------------------------------------- plan

def cost_effectiveness(sp: float, cost: float) -> float:
    return (1.0 - sp) / cost


def order_predicates(sp: Sequence[float], cost: Sequence[float]) -> List[int]:
    """Predicate ids sorted by (1 - sp) / cost descending; stable on ties."""
    ce = [cost_effectiveness(s, c) for s, c in zip(sp, cost)]
    return sorted(range(len(sp)), key=lambda p: -ce[p])


class Node:
    def __init__(self, pred: int = -1, parent=None):
        self.pred = pred
        self.parent = parent
        self.children: List["Node"] = []
        self.rules: List[int] = []      # rules whose path ends here
        self.score = 0.0


def build_tree(rules: Sequence[Sequence[int]], order: Sequence[int]) -> Tuple[Node, List[List[Node]]]:
    """Insert each rule's predicates, sorted by `order`, re-using child edges.
    Returns the root and, per rule, its root-to-leaf node path."""
    rank = {p: r for r, p in enumerate(order)}
    root = Node()
    paths = []
    for r, preds in enumerate(rules):
        ps = sorted(set(preds), key=lambda p: rank[p])
        node = root
        path = []
        for p in ps:
            nxt = None
            for c in node.children:
                if c.pred == p:
                    nxt = c
                    break
            if nxt is None:
                nxt = Node(p, node)
                node.children.append(nxt)
            node = nxt
            path.append(node)
        node.rules.append(r)
        paths.append(path)
    return root, paths


def witness_probability(rule: Sequence[int], sp: Sequence[float]) -> float:
    w = 1.0
    for p in sorted(set(rule)):
        w *= sp[p]
    return w


def score_edges(rules, paths, sp) -> None:
    wp = [witness_probability(r, sp) for r in rules]
    for r, path in enumerate(paths):
        for node in path:  # the edge (parent, node)
            node.score = max(node.score, wp[r])


def dfs_rules(root: Node) -> List[int]:
    out: List[int] = []

    def visit(n: Node):
        out.extend(sorted(n.rules))
        kids = sorted(range(len(n.children)), key=lambda c: -n.children[c].score)
        for c in kids:
            visit(n.children[c])

    visit(root)
    return out


def sequential_path(rules: Sequence[Sequence[int]], sp: Sequence[float], cost: Sequence[float]):
    """The flattened plan: [(rule id, [pred ids root-to-leaf]), ...] in DFS order."""
    order = order_predicates(sp, cost)
    root, paths = build_tree(rules, order)
    score_edges(rules, paths, sp)
    seq = dfs_rules(root)
    return [(r, [n.pred for n in paths[r]]) for r in seq], root, paths

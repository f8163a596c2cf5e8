"""CPU oracle for rule-based blocking -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library
(`paper_2410_04349_amd`) and never imports it.

  * `hboracle.cpp` -- the matched-pair set Ca(D, Delta) by the definition of
    Section 2 ("Rule-based blocking"), evaluated naively as at the start of
    Section 4: full Levenshtein table, std::set q-gram sets, integer
    Jaccard test, 128-bit range test.
  * `epg.py` -- the execution-plan generator arithmetic of Section 4.2
    (cost-effectiveness ordering, execution tree, witness probability, edge
    scores, DFS order) and the LSH selectivity estimate.
  * `pairnet.py` -- the per-pair cost network's inputs and estimate of
    Section 4.2 ("Evaluation cost", "Estimated cost"): sampled pairs of
    D x D, their features, and norm(sum of the network's estimates).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hboracle.cpp")
_LIB = os.path.join(_HERE, "libhboracle.so")

_TYPES = {"string": 0, "categorical": 1, "int64": 2}
_OPS = {"eq": 0, "ed": 1, "jaccard": 2, "absdiff": 3, "eq_const": 4, "eq_cross": 5, "ed_cross": 6,
        "jaccard_cross": 7, "contain": 8}


class _Col(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("offsets", ctypes.c_void_p), ("data", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("valid", ctypes.c_void_p)]


class _Pred(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("attr", ctypes.c_uint32), ("k", ctypes.c_int64),
                ("q", ctypes.c_uint32), ("num", ctypes.c_uint32), ("den", ctypes.c_uint32),
                ("d", ctypes.c_int64), ("attr_b", ctypes.c_uint32), ("side", ctypes.c_int32),
                ("c", ctypes.c_int64)]


def build_lib(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_lib())
        P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        # full prototypes: 64-bit sizes must not travel as C ints
        for name, res, args in (
                ("ora_levenshtein", ctypes.c_int64, [P, U64, P, U64]),
                ("ora_qgram_stats", None, [P, U64, P, U64, U32, P, P, P]),
                ("ora_jaccard_ge", I, [P, U64, P, U64, U32, U32, U32]),
                ("ora_sat", I, [P, P, U64, U64]),
                ("ora_rule_witness", I, [P, U32, P, U64, U64]),
                ("ora_blocking", ctypes.c_int64, [P, U32, U64, U32, P, P, I, I, P, U64]),
                ("ora_candidate_count", ctypes.c_int64, [P, U64, U32, P, P]),
                ("ora_eval_pairs", I, [P, U64, U32, P, P, P, U64, I, P]),
                ("ora_ordered", I, [U32, P, P])):
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class _Marshal:
    """Keeps the numpy buffers alive while the C structs point at them."""

    def __init__(self, rel, rules):
        self.keep = []
        self.cols = (_Col * max(1, len(rel.columns)))()
        for k, c in enumerate(rel.columns):
            arrs = []
            for a in (c.offsets, c.data, c.values, c.valid):
                if a is not None:
                    a = np.ascontiguousarray(a)
                arrs.append(a)
            self.keep.extend(arrs)
            off, data, vals, valid = arrs
            if data is not None and data.size == 0:
                data = np.zeros(1, np.uint8)
                self.keep.append(data)
            self.cols[k] = _Col(_TYPES[c.type], _ptr(off).value if off is not None else None,
                                _ptr(data).value if data is not None else None,
                                _ptr(vals).value if vals is not None else None,
                                _ptr(valid).value if valid is not None else None)
        flat = [p for r in rules for p in r]
        self.n_rules = len(rules)
        self.rule_len = (ctypes.c_uint32 * max(1, len(rules)))(*[len(r) for r in rules])
        self.preds = (_Pred * max(1, len(flat)))()
        for x, p in enumerate(flat):
            self.preds[x] = to_cpred(p)


def to_cpred(p):
    return _Pred(_OPS[p.op], p.attr, p.k, p.q, p.num, p.den, p.d, getattr(p, "attr_b", 0),
                 getattr(p, "side", 0), getattr(p, "c", 0))


def levenshtein(a: bytes, b: bytes) -> int:
    return int(_load().ora_levenshtein(a, len(a), b, len(b)))


def qgram_stats(a: bytes, b: bytes, q: int):
    """(|G_q(a)|, |G_q(a) & G_q(b)|, |G_q(a) | G_q(b)|)"""
    sa, i, u = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _load().ora_qgram_stats(a, len(a), b, len(b), q, ctypes.byref(sa), ctypes.byref(i), ctypes.byref(u))
    return sa.value, i.value, u.value


def jaccard_ge(a: bytes, b: bytes, q: int, num: int, den: int) -> bool:
    return bool(_load().ora_jaccard_ge(a, len(a), b, len(b), q, num, den))


def sat(rel, pred, i: int, j: int) -> bool:
    m = _Marshal(rel, [[pred]])
    return bool(_load().ora_sat(m.cols, ctypes.byref(m.preds[0]), i, j))


def rule_witness(rel, rule, i: int, j: int) -> bool:
    m = _Marshal(rel, [rule])
    return bool(_load().ora_rule_witness(m.cols, len(rule), m.preds, i, j))


def ordered(rules) -> bool:
    """True if some predicate tells t from s (t.A = c, s.A = c, or t.A = s.B
    or t.A ~ s.B over two different attributes): Ca then lists ordered
    pairs."""
    flat = [p for r in rules for p in r]
    lens = (ctypes.c_uint32 * max(1, len(rules)))(*[len(r) for r in rules])
    preds = (_Pred * max(1, len(flat)))(*[to_cpred(p) for p in flat])
    return bool(_load().ora_ordered(len(rules), lens, preds))


def blocking(rel, rules, mode: str = "blocked", threads: int = 1) -> np.ndarray:
    """Ca(D, Delta): sorted uint64 array of (i << 32) | j (t bound to row i,
    s to row j); i < j unless the rule set is ordered."""
    m = _Marshal(rel, rules)
    md = {"blocked": 0, "full": 1}[mode]
    lib = _load()
    cap = 1 << 16
    while True:
        out = np.zeros(cap, dtype=np.uint64)
        n = lib.ora_blocking(m.cols, len(rel.columns), rel.n_rows, m.n_rules, m.rule_len, m.preds,
                             md, threads, _ptr(out), cap)
        if n == -2:
            raise ValueError("a rule has no equality on a categorical/int64 key")
        if n <= cap:
            return out[:n].copy()
        cap = int(n)


def candidate_count(rel, rules) -> int:
    m = _Marshal(rel, rules)
    n = _load().ora_candidate_count(m.cols, rel.n_rows, m.n_rules, m.rule_len, m.preds)
    if n == -2:
        raise ValueError("a rule has no equality on a categorical/int64 key")
    return int(n)


def eval_pairs(rel, rules, pairs: np.ndarray, threads: int = 1) -> np.ndarray:
    """Boolean array: pairs[x] (packed (i << 32) | j) is in Ca(D, Delta)."""
    m = _Marshal(rel, rules)
    pairs = np.ascontiguousarray(pairs, dtype=np.uint64)
    flags = np.zeros(max(1, len(pairs)), dtype=np.uint8)
    _load().ora_eval_pairs(m.cols, rel.n_rows, m.n_rules, m.rule_len, m.preds, _ptr(pairs),
                           len(pairs), threads, _ptr(flags))
    return flags[: len(pairs)].astype(bool)

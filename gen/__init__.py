"""Seeded synthetic relations and rule sets (input generators only).

This package draws inputs; it holds none of the blocking method's
arithmetic.  Both the CPU oracle and the GPU library consume what it
produces, and neither is imported here.

A relation is a list of typed columns:
  * ``string``      -- ``offsets`` (uint64, n+1) and ``data`` (uint8 bytes)
  * ``categorical`` -- ``values`` (int64 codes)
  * ``int64``       -- ``values`` (int64)
each with an optional LSB-first validity bitmap ``valid`` (None = all valid).

A rule is a list of predicates (conjunction); a rule set is a list of rules
(disjunction), following the matching-dependency form of Section 2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hbgen.c")
_LIB = os.path.join(_HERE, "libhbgen.so")

STRING, CATEGORICAL, INT64 = "string", "categorical", "int64"
EQ, ED, JACCARD, ABSDIFF = "eq", "ed", "jaccard", "absdiff"
EQ_CONST, EQ_CROSS = "eq_const", "eq_cross"   # t.A = c (side 0) / s.A = c (side 1); t.A = s.B
ED_CROSS = "ed_cross"                           # edit distance from t.A to s.B <= k
JACCARD_CROSS = "jaccard_cross"                 # q-gram Jaccard of t.A and s.B >= num / den
CONTAIN = "contain"                             # share of t.A's q-grams found in s.B's >= num / den (asymmetric)


@dataclass
class Column:
    name: str
    type: str
    offsets: Optional[np.ndarray] = None
    data: Optional[np.ndarray] = None
    values: Optional[np.ndarray] = None
    valid: Optional[np.ndarray] = None

    def is_valid(self, i: int) -> bool:
        if self.valid is None:
            return True
        return bool((self.valid[i >> 3] >> (i & 7)) & 1)

    def get(self, i: int):
        if self.type == STRING:
            return bytes(self.data[self.offsets[i]:self.offsets[i + 1]])
        return int(self.values[i])


@dataclass
class Relation:
    columns: List[Column]
    n_rows: int
    dup_src: Optional[np.ndarray] = None

    def col(self, name: str) -> int:
        for k, c in enumerate(self.columns):
            if c.name == name:
                return k
        raise KeyError(name)

    def take(self, rows: Sequence[int]) -> "Relation":
        """Sub-relation holding `rows` in the given order (row i of the result
        is row rows[i] of self)."""
        rows = np.asarray(rows, dtype=np.int64)
        cols = []
        for c in self.columns:
            valid = None
            if c.valid is not None:
                bits = np.unpackbits(c.valid, bitorder="little")[rows]
                valid = pack_bits(bits)
            if c.type == STRING:
                starts = c.offsets[rows].astype(np.int64)
                ends = c.offsets[rows + 1].astype(np.int64)
                lens = ends - starts
                offs = np.zeros(len(rows) + 1, dtype=np.uint64)
                np.cumsum(lens, out=offs[1:])
                total = int(lens.sum())
                if total:
                    # byte k of the result comes from starts[row of k] + (k - offs[row of k])
                    owner = np.repeat(np.arange(len(rows)), lens)
                    idx = starts[owner] + (np.arange(total) - offs[:-1].astype(np.int64)[owner])
                    data = c.data[idx].copy()
                else:
                    data = np.zeros(0, np.uint8)
                cols.append(Column(c.name, c.type, offsets=offs, data=data, valid=valid))
            else:
                cols.append(Column(c.name, c.type, values=c.values[rows].copy(), valid=valid))
        dup = None
        if self.dup_src is not None:
            dup = np.full(len(rows), -1, dtype=np.int64)
        return Relation(cols, len(rows), dup)


def entity_ids(rel: Relation) -> np.ndarray:
    """Ground-truth entity of every row: a base tuple is its own entity and
    a generated duplicate belongs to its source's (links followed to the
    root).  Relations without duplicate links give one entity per row."""
    n = rel.n_rows
    ent = np.arange(n, dtype=np.int64)
    if rel.dup_src is None:
        return ent
    src = np.asarray(rel.dup_src, dtype=np.int64)
    for _ in range(64):   # links point at earlier generations; a few hops reach the root
        nxt = np.where(src[ent] >= 0, src[ent], ent)
        if np.array_equal(nxt, ent):
            break
        ent = nxt
    return ent


def true_pairs(rel: Relation) -> np.ndarray:
    """Every pair (i, j), i < j, of rows of one ground-truth entity, packed
    (i << 32) | j and sorted (the layout of the library's result)."""
    ent = entity_ids(rel)
    order = np.lexsort((np.arange(len(ent)), ent))   # by entity, rows ascending within
    e = ent[order]
    starts = np.flatnonzero(np.r_[True, e[1:] != e[:-1]])
    sizes = np.diff(np.r_[starts, len(e)])
    out = []
    for m in np.unique(sizes[sizes >= 2]):   # every group of one size at once
        base = starts[sizes == m]
        a, b = np.triu_indices(int(m), k=1)
        ra = order[base[:, None] + a[None, :]].astype(np.uint64).ravel()
        rb = order[base[:, None] + b[None, :]].astype(np.uint64).ravel()
        out.append((ra << np.uint64(32)) | rb)
    if not out:
        return np.zeros(0, dtype=np.uint64)
    return np.sort(np.concatenate(out))


@dataclass(frozen=True)
class Pred:
    op: str
    attr: int
    k: int = 0          # ED threshold (distance <= k)
    q: int = 0          # Jaccard q-gram length
    num: int = 0        # Jaccard threshold num/den
    den: int = 1
    d: int = 0          # ABSDIFF threshold |a-b| <= d
    attr_b: int = 0     # EQ_CROSS, ED_CROSS, JACCARD_CROSS, CONTAIN: the attribute B of t.A = s.B, t.A ~ s.B
    side: int = 0       # EQ_CONST: 0 for t.A = c, 1 for s.A = c
    c: int = 0          # EQ_CONST: the constant


def pack_bits(bits: np.ndarray) -> np.ndarray:
    return np.packbits(np.asarray(bits, dtype=np.uint8), bitorder="little")


def string_column(name: str, strings: Sequence[Optional[bytes]]) -> Column:
    """Build a string column from Python bytes; None marks a missing value."""
    lens = [0 if s is None else len(s) for s in strings]
    offs = np.zeros(len(strings) + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    data = np.frombuffer(b"".join(s or b"" for s in strings), dtype=np.uint8).copy()
    valid = None
    if any(s is None for s in strings):
        valid = pack_bits([0 if s is None else 1 for s in strings])
    return Column(name, STRING, offsets=offs, data=data, valid=valid)


def int_column(name: str, values: Sequence[Optional[int]], type_: str = INT64) -> Column:
    vals = np.array([0 if v is None else v for v in values], dtype=np.int64)
    valid = None
    if any(v is None for v in values):
        valid = pack_bits([0 if v is None else 1 for v in values])
    return Column(name, type_, values=vals, valid=valid)


# ---------------------------------------------------------------- C generator

class _Attr(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("alphabet", ctypes.c_int32),
                ("min_len", ctypes.c_uint32), ("max_len", ctypes.c_uint32),
                ("editable", ctypes.c_int32), ("zipf_s", ctypes.c_double),
                ("n_values", ctypes.c_uint32), ("cap", ctypes.c_uint32),
                ("lo", ctypes.c_int64), ("hi", ctypes.c_int64),
                ("int_p", ctypes.c_double), ("int_d", ctypes.c_int64),
                ("dep", ctypes.c_int32), ("dep_p", ctypes.c_double)]


class _Spec(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_base", ctypes.c_uint32),
                ("n_dup", ctypes.c_uint32), ("edit_min", ctypes.c_uint32),
                ("edit_max", ctypes.c_uint32), ("n_attrs", ctypes.c_uint32)]


class _Out(ctypes.Structure):
    _fields_ = [("offsets", ctypes.c_void_p), ("bytes", ctypes.c_void_p),
                ("bytes_cap", ctypes.c_uint64), ("values", ctypes.c_void_p)]


_KIND = {"string": 0, "words": 1, "zipf": 2, "codes": 3, "int": 4, "keyed": 5}
_STRING_KINDS = ("string", "words", "keyed")


def build_lib(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build_lib())
        _lib.hbgen_generate.restype = ctypes.c_int
    return _lib


@dataclass
class AttrSpec:
    name: str
    kind: str                     # string | words | zipf | codes | int | keyed
    alphabet: int = 0
    min_len: int = 0
    max_len: int = 0
    editable: bool = True
    zipf_s: float = 1.0
    n_values: int = 0
    cap: int = 0
    lo: int = 0
    hi: int = 0
    int_p: float = 0.0
    int_d: int = 0
    dep: int = -1                 # keyed: index of the key attribute it follows
    dep_p: float = 0.0            # keyed: probability that a key code is pinned


def generate(seed: int, n_base: int, n_dup: int, attrs: Sequence[AttrSpec],
             edit_min: int = 1, edit_max: int = 2) -> Relation:
    lib = _load()
    n = n_base + n_dup
    na = len(attrs)
    carr = (_Attr * na)()
    outs = (_Out * na)()
    keep = []
    for a, s in enumerate(attrs):
        carr[a] = _Attr(_KIND[s.kind], s.alphabet, s.min_len, s.max_len, int(s.editable),
                        s.zipf_s, s.n_values, s.cap, s.lo, s.hi, s.int_p, s.int_d, s.dep, s.dep_p)
        if s.kind in _STRING_KINDS:
            offs = np.zeros(n + 1, dtype=np.uint64)
            cap = n * (s.max_len + edit_max) + 1
            data = np.zeros(cap, dtype=np.uint8)
            outs[a] = _Out(offs.ctypes.data, data.ctypes.data, cap, None)
            keep.append((offs, data))
        else:
            vals = np.zeros(n, dtype=np.int64)
            outs[a] = _Out(None, None, 0, vals.ctypes.data)
            keep.append((vals,))
    dup = np.zeros(n, dtype=np.int64)
    used = np.zeros(na, dtype=np.uint64)
    spec = _Spec(seed, n_base, n_dup, edit_min, edit_max, na)
    rc = lib.hbgen_generate(ctypes.byref(spec), carr, outs, ctypes.c_void_p(dup.ctypes.data),
                            ctypes.c_void_p(used.ctypes.data))
    if rc != 0:
        raise RuntimeError(f"hbgen_generate failed with code {rc}")
    cols = []
    for a, s in enumerate(attrs):
        if s.kind in _STRING_KINDS:
            offs, data = keep[a]
            cols.append(Column(s.name, STRING, offsets=offs, data=data[: int(used[a])].copy()))
        else:
            t = INT64 if s.kind == "int" else CATEGORICAL
            cols.append(Column(s.name, t, values=keep[a][0]))
    return Relation(cols, n, dup)

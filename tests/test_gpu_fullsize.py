"""Parity at full workload sizes.  Every emitted pair is checked by the
oracle (soundness).  Whole blocks are checked exhaustively: the result
restricted to the rows of the largest blocks of each key (several 64 x 64
tiles each), or of a seeded draw of blocks, equals the oracle's Ca of the
sub-relation on those rows (Ca is defined pairwise, so a row subset's
result is the full result restricted to it).  Where the oracle enumerated
the whole workload on a host CPU (tests/golden/fullsize_digests.json,
written by tests/golden/make_fullsize_digests.py), the sorted pair list's
count and sha256 equal the oracle's.  A seeded sample of candidate pairs,
drawn uniformly over each key's candidate pairs, plus every (duplicate,
source) pair, is checked for membership; the candidate count is checked
against the closed form.  Runs both plans, the learned one with a freshly
trained model, in the launch configuration the benchmark times."""
import hashlib
import importlib.util
import json
import os

import numpy as np
import pytest

import oracle
from gen import EQ, STRING, workloads
from learned_util import train_model

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_04349_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(hb):
    c = hb.hb_create(0, allocator="torch")
    hb.hb_set_learned_min_saving(c, 0.0)   # every per-block plan kept: their parity
    hb.hb_set_pack_small_blocks(c, True)   # the long-title blocks packed into shared tiles
    assert np.isfinite(train_model(hb, c))
    yield c
    c.close()


def key_attrs(rel, rules):
    """Each rule's blocking key: its first equality on a categorical or
    int64 attribute; distinct keys in first-appearance order."""
    keys = []
    for r in rules:
        k = next(p.attr for p in r if p.op == EQ and rel.columns[p.attr].type != STRING)
        if k not in keys:
            keys.append(k)
    return keys


def valid_mask(col, n):
    if col.valid is None:
        return np.ones(n, dtype=bool)
    return np.unpackbits(col.valid, bitorder="little")[:n].astype(bool)


def sample_pairs(rel, keys, n_sample, seed):
    """Uniform sample of each key's candidate pairs (i < j) plus every
    co-blocked (duplicate, source) pair, packed (i << 32) | j, unique."""
    r = np.random.default_rng(seed)
    out = []
    for key in keys:
        vals = rel.columns[key].values
        ok = valid_mask(rel.columns[key], rel.n_rows)
        rows = np.flatnonzero(ok)
        order = rows[np.argsort(vals[rows], kind="stable")]
        v = vals[order]
        starts = np.flatnonzero(np.r_[True, v[1:] != v[:-1]])
        sizes = np.diff(np.r_[starts, len(v)])
        w = sizes * (sizes - 1) / 2.0
        if w.sum() == 0:
            continue
        b = r.choice(len(sizes), size=n_sample, p=w / w.sum())
        a = r.integers(0, sizes[b])
        c = r.integers(0, sizes[b] - 1)
        c = np.where(c >= a, c + 1, c)
        i = order[starts[b] + a]
        j = order[starts[b] + c]
        lo, hi = np.minimum(i, j), np.maximum(i, j)
        out.append((lo.astype(np.uint64) << np.uint64(32)) | hi.astype(np.uint64))
        d = np.flatnonzero(rel.dup_src >= 0)
        s = rel.dup_src[d]
        same = ok[d] & ok[s] & (vals[d] == vals[s])
        d, s = d[same], s[same]
        lo, hi = np.minimum(d, s), np.maximum(d, s)
        out.append((lo.astype(np.uint64) << np.uint64(32)) | hi.astype(np.uint64))
    return np.unique(np.concatenate(out))


def closed_form_single_key(rel, key):
    vals = rel.columns[key].values[valid_mask(rel.columns[key], rel.n_rows)]
    _, c = np.unique(vals, return_counts=True)
    return int((c * (c - 1) // 2).sum())


def closed_form_keys(rel, keys):
    """Distinct pairs sharing at least one key value, by inclusion-exclusion
    over the keys' composite groups (numpy; the oracle's exact count
    enumerates pairs and does not fit memory at 10M tuples)."""
    n = rel.n_rows
    total = 0
    for m in range(1, 1 << len(keys)):
        sub = [k for x, k in enumerate(keys) if m >> x & 1]
        ok = np.ones(n, dtype=bool)
        for k in sub:
            ok &= valid_mask(rel.columns[k], n)
        cols = np.stack([rel.columns[k].values[ok] for k in sub], axis=1)
        _, c = np.unique(cols, axis=0, return_counts=True)
        pairs = int((c.astype(np.int64) * (c - 1) // 2).sum())
        total += pairs if len(sub) % 2 == 1 else -pairs
    return total


def eval_in_chunks(rel, rules, pairs, chunk=200_000):
    """oracle.eval_pairs on sub-relations of the rows each chunk of pairs
    touches (the oracle marshals its whole input relation, which does not
    fit memory at 10M tuples); pair order is kept."""
    out = np.zeros(len(pairs), dtype=bool)
    for a in range(0, len(pairs), chunk):
        p = pairs[a:a + chunk]
        i, j = p >> np.uint64(32), p & np.uint64(0xFFFFFFFF)
        rows = np.unique(np.concatenate([i, j]))
        sub = rel.take(rows.astype(np.int64))
        ni = np.searchsorted(rows, i).astype(np.uint64)
        nj = np.searchsorted(rows, j).astype(np.uint64)
        out[a:a + chunk] = oracle.eval_pairs(sub, rules, (ni << np.uint64(32)) | nj, threads=16)
    return out


def _digests():
    spec = importlib.util.spec_from_file_location("make_fullsize_digests",
                                                  os.path.join(GOLDEN, "make_fullsize_digests.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    path = os.path.join(GOLDEN, "fullsize_digests.json")
    table = {}
    if os.path.exists(path):
        with open(path) as fh:
            table = json.load(fh)
    return mod, table


def sha256_pairs(p):
    return hashlib.sha256(np.ascontiguousarray(p, dtype="<u8").tobytes()).hexdigest()


def check_digest(name, rel, got):
    """The whole result against the oracle's, by count and sha256 of the
    sorted packed list (when the oracle's full enumeration is on file), and
    the result restricted to each block set on file against the oracle's
    Ca of that sub-relation.  Returns whether the full enumeration was on
    file."""
    mod, table = _digests()
    full = name in table
    if full:
        rec = table[name]
        assert mod.relation_digest(rel) == rec["relation_sha256"], "the generator's output changed: rerun the script"
        assert len(got) == rec["matched_pairs"]
        assert sha256_pairs(got) == rec["pairs_sha256"]
        print(f"[gpu-case] {name}: all {len(got)} pairs equal the oracle's full enumeration (sha256)", flush=True)
    for bname, rec in sorted(table.items()):
        if not bname.startswith(name + "/"):
            continue
        rows = mod.digest_rows(rel, rec["blocks"])
        assert mod.rows_digest(rows) == rec["rows_sha256"]
        mapped = restrict(got, rows)
        assert len(mapped) == rec["matched_pairs"] and sha256_pairs(mapped) == rec["pairs_sha256"], bname
        print(f"[gpu-case] {bname}: {len(rows)} rows, {len(mapped)} matches equal the oracle's (sha256)", flush=True)
    return full


def block_rows(rel, key, largest=0, draw=0, seed=0, max_size=None):
    """Rows of whole blocks of `key`: its `largest` largest blocks and a
    seeded draw of `draw` other blocks of at least two (and at most
    `max_size`) rows."""
    vals = rel.columns[key].values
    ok = valid_mask(rel.columns[key], rel.n_rows)
    idx = np.flatnonzero(ok)
    uniq, inv, cnt = np.unique(vals[idx], return_inverse=True, return_counts=True)
    order = np.argsort(-cnt, kind="stable")
    chosen = list(order[:largest])
    rest = order[largest:]
    rest = rest[(cnt[rest] >= 2) & (cnt[rest] <= (max_size or cnt.max()))]
    if draw and len(rest):
        chosen += list(np.random.default_rng(seed).choice(rest, size=min(draw, len(rest)), replace=False))
    return idx[np.isin(inv, np.asarray(chosen, dtype=np.int64))]


def restrict(got, rows):
    """The pairs of `got` with both rows in `rows` (ascending), renumbered
    to positions in `rows`; the order is kept."""
    i, j = got >> np.uint64(32), got & np.uint64(0xFFFFFFFF)
    inside = np.isin(i, rows) & np.isin(j, rows)
    mi = np.searchsorted(rows, i[inside]).astype(np.uint64)
    mj = np.searchsorted(rows, j[inside]).astype(np.uint64)
    return (mi << np.uint64(32)) | mj


def check_blocks(rel, rules, got, rows):
    """Ca(D) restricted to pairs of `rows` equals the oracle's Ca of the
    sub-relation on `rows`, element by element."""
    rows = np.unique(rows)
    want = oracle.blocking(rel.take(rows), rules, threads=16)
    mapped = restrict(got, rows)
    assert np.array_equal(mapped, want), (len(mapped), len(want))
    print(f"[gpu-case] whole blocks: {len(rows)} rows, {len(want)} matches, equal to the oracle's", flush=True)


def check(hb, ctx, rel, rules, n_sample, seed, plans=("heuristic", "learned"), max_sample=None, ordered=False,
          name=None, blocks=None):
    rid = hb.hb_load_relation(ctx, rel.columns, rel.n_rows)
    rs = hb.hb_compile_rules(ctx, rid, rules)
    n_cand = hb.hb_partition(ctx, rid, rs)
    outs = {}
    for plan in plans:
        print(f"[gpu-case] {rel.n_rows} tuples, plan {plan}", flush=True)
        outs[plan] = hb.hb_match(ctx, rid, rs, plan)
    hb.hb_release_relation(ctx, rid)
    keys = key_attrs(rel, rules)
    if len(keys) == 1:
        assert n_cand == closed_form_single_key(rel, keys[0])
    else:
        assert n_cand == closed_form_keys(rel, keys)
    got = outs[plans[0]]
    for plan in plans[1:]:
        assert np.array_equal(outs[plan], got), plan
    assert np.all(got[:-1] < got[1:])
    big = rel.n_rows > 2_000_000
    ev = (lambda p: eval_in_chunks(rel, rules, p)) if big else (lambda p: oracle.eval_pairs(rel, rules, p, threads=16))
    assert np.all(ev(got))
    sample = sample_pairs(rel, keys, n_sample, seed)
    if max_sample is not None and len(sample) > max_sample:
        sample = np.sort(np.random.default_rng(seed).choice(sample, size=max_sample, replace=False))
    if ordered:   # both valuations of every sampled pair
        sample = np.unique(np.concatenate([sample, (sample << np.uint64(32)) | (sample >> np.uint64(32))]))
    want = ev(sample)
    have = np.isin(sample, got)
    assert np.array_equal(have, want), int(np.sum(have != want))
    print(f"[gpu-case] {len(got)} matches all confirmed; {len(sample)} sampled pairs, "
          f"{int(want.sum())} matching, agree", flush=True)
    for spec in blocks or ():
        check_blocks(rel, rules, got, np.concatenate([block_rows(rel, **b) for b in spec]))
    if name is not None and not check_digest(name, rel, got):
        print(f"[gpu-case] {name}: no full oracle enumeration on file (whole blocks and samples only)", flush=True)


def test_plain_1m_full_size(hb, ctx):
    """Whole result against the oracle's full enumeration; the two largest
    blocks (about 5,000 rows, 79 tiles wide) exhaustively."""
    rel, rules = workloads.plain_1m()
    check(hb, ctx, rel, rules, 300_000, 1, name="plain_1m",
          blocks=[[{"key": 3, "largest": 2}]])


def test_long_titles_5m_full_size(hb, ctx):
    """Whole result against the oracle's full enumeration; a seeded draw of
    4,000 whole brand blocks exhaustively."""
    rel, rules = workloads.long_titles_5m()
    check(hb, ctx, rel, rules, 200_000, 2, name="long_titles_5m",
          blocks=[[{"key": 0, "largest": 1, "draw": 4000, "seed": 5}]])


def test_plain_1m_ordered_full_size(hb, ctx):
    """plain_1m under a rule set with t.i1 = 7 (ordered output), in the
    benchmark's grammar leg: every listed ordered pair confirmed by the
    oracle's valuation, both orders of a candidate sample checked."""
    rel, _ = workloads.plain_1m()
    check(hb, ctx, rel, workloads.plain_1m_ordered_rules(), 150_000, 4, plans=("heuristic",), ordered=True)


def test_learned_10m_full_size(hb, ctx):
    """The two-key, 20-rule, 10M-tuple workload: candidate count against
    the inclusion-exclusion closed form, every emitted pair confirmed by the
    oracle, a sample of both keys' candidate pairs checked, both plans
    equal; a seeded draw of whole blocks of each key against the oracle
    here, and the largest block of each key (about 5,000 rows, where this
    oracle evaluates some 10^4 pairs per second) against its result on
    file."""
    rel, rules = workloads.learned_10m()
    check(hb, ctx, rel, rules, 150_000, 3, max_sample=300_000, name="learned_10m",
          blocks=[[{"key": 4, "draw": 300, "seed": 6, "max_size": 150},
                   {"key": 5, "draw": 300, "seed": 7, "max_size": 150}]])

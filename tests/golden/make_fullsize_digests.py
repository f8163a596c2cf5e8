#!/usr/bin/env python3
"""Write tests/golden/fullsize_digests.json: for each full-size workload the
oracle can enumerate on a host CPU, the whole of Ca(D, Delta) computed by
the oracle (every candidate pair of every key block, Section 2 "Rule-based
blocking"), stored as its pair count and the sha256 of the sorted packed
u64 list (little-endian), beside a sha256 of the generated relation so a
change of the generator is told apart from a change of the result.

Calls only the seeded generators (gen/) and the oracle (oracle/).  The
10M-tuple two-key workload (about 4e10 candidate pairs) is out of the
oracle's reach and is not here.

For workloads out of the oracle's reach as a whole, entries named
"<workload>/<blocks>" hold the oracle's Ca of the sub-relation on the rows
of whole key blocks (Ca is defined pairwise, so it equals the full result
restricted to those rows): the rows' sha256, the pair count and the sha256
of the sorted list renumbered to positions among the rows.

    python tests/golden/make_fullsize_digests.py [--threads N] [entry ...]
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from gen import workloads  # noqa: E402

OUT = os.path.join(HERE, "fullsize_digests.json")
LOADERS = {"plain_1m": workloads.plain_1m, "long_titles_5m": workloads.long_titles_5m,
           "learned_10m": workloads.learned_10m}
# block sets: the largest block of each key of the 10M two-key workload
BLOCK_SETS = {
    "learned_10m/largest_k1": ("learned_10m", [{"key": 4, "largest": 1}]),
    "learned_10m/largest_k2": ("learned_10m", [{"key": 5, "largest": 1}]),
}
FULL = ("plain_1m", "long_titles_5m")


def digest_rows(rel, blocks):
    """Ascending rows of the given whole blocks: per entry, the `largest`
    largest value groups of attribute `key` (ties by value order)."""
    out = []
    for b in blocks:
        col = rel.columns[b["key"]]
        ok = np.ones(rel.n_rows, dtype=bool)
        if col.valid is not None:
            ok = np.unpackbits(col.valid, bitorder="little")[:rel.n_rows].astype(bool)
        idx = np.flatnonzero(ok)
        _, inv, cnt = np.unique(col.values[idx], return_inverse=True, return_counts=True)
        top = np.argsort(-cnt, kind="stable")[:b["largest"]]
        out.append(idx[np.isin(inv, top)])
    return np.unique(np.concatenate(out))


def rows_digest(rows) -> str:
    return hashlib.sha256(np.ascontiguousarray(rows, dtype="<i8").tobytes()).hexdigest()


def relation_digest(rel) -> str:
    """sha256 over every column's buffers in order (type, offsets, bytes,
    values, validity)."""
    h = hashlib.sha256()
    h.update(str(rel.n_rows).encode())
    for c in rel.columns:
        h.update(c.type.encode())
        for a in (c.offsets, c.data, c.values, c.valid):
            h.update(b"-" if a is None else np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def pairs_digest(pairs: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(pairs, dtype="<u8").tobytes()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("entries", nargs="*", default=list(FULL) + list(BLOCK_SETS))
    args = ap.parse_args()
    for name in args.entries:
        if name in BLOCK_SETS:
            wl, blocks = BLOCK_SETS[name]
            rel, rules = LOADERS[wl]()
            rows = digest_rows(rel, blocks)
            t0 = time.perf_counter()
            pairs = oracle.blocking(rel.take(rows), rules, threads=args.threads)
            rec = {"blocks": blocks, "rows": int(len(rows)), "rows_sha256": rows_digest(rows),
                   "relation_sha256": relation_digest(rel)}
        else:
            rel, rules = LOADERS[name]()
            t0 = time.perf_counter()
            pairs = oracle.blocking(rel, rules, threads=args.threads)
            rec = {"n_rows": int(rel.n_rows), "relation_sha256": relation_digest(rel)}
        dt = time.perf_counter() - t0
        rec.update({"matched_pairs": int(len(pairs)), "pairs_sha256": pairs_digest(pairs),
                    "oracle_seconds": round(dt, 1), "oracle_threads": args.threads})
        print(name, rec, flush=True)
        # re-read: other runs of this script may have written entries meanwhile
        table = {}
        if os.path.exists(OUT):
            with open(OUT) as fh:
                table = json.load(fh)
        table[name] = rec
        with open(OUT + ".tmp", "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
            fh.write("\n")
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()

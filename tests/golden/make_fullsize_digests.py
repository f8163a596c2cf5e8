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

    python tests/golden/make_fullsize_digests.py [--threads N] [workload ...]
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
LOADERS = {"plain_1m": workloads.plain_1m, "long_titles_5m": workloads.long_titles_5m}


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
    ap.add_argument("workloads", nargs="*", default=list(LOADERS))
    args = ap.parse_args()
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            table = json.load(fh)
    for name in args.workloads:
        rel, rules = LOADERS[name]()
        t0 = time.perf_counter()
        pairs = oracle.blocking(rel, rules, threads=args.threads)
        dt = time.perf_counter() - t0
        table[name] = {
            "n_rows": int(rel.n_rows),
            "relation_sha256": relation_digest(rel),
            "matched_pairs": int(len(pairs)),
            "pairs_sha256": pairs_digest(pairs),
            "oracle_seconds": round(dt, 1),
            "oracle_threads": args.threads,
        }
        print(name, table[name], flush=True)
        with open(OUT, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
            fh.write("\n")


if __name__ == "__main__":
    main()

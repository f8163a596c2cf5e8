"""Quality of a blocking result against synthetic ground truth (a report on
the output, computed on the host; not a step of the matching path).

The measures are the paper's (Section 6, "Measurements"): precision = the
share of identified pairs that are true matches, recall = the share of true
matches that were identified, F1 = their harmonic mean, and the candidate
set size ratio CSSR = |Ca(P)| / (|P| x |P|) -- the portion of all tuple
pairs left for a matcher, smaller being better.
"""
import numpy as np


def quality(pairs, truth, n_rows: int) -> dict:
    """pairs, truth: packed (i << 32) | j result lists (i < j, any order,
    no repeats), e.g. hb_match's output and gen.true_pairs(relation)."""
    pairs = np.unique(np.asarray(pairs, dtype=np.uint64))
    truth = np.unique(np.asarray(truth, dtype=np.uint64))
    hit = int(np.intersect1d(pairs, truth, assume_unique=True).size)
    prec = hit / pairs.size if pairs.size else 1.0
    rec = hit / truth.size if truth.size else 1.0
    f1 = 2.0 * prec * rec / (prec + rec) if prec + rec > 0 else 0.0
    return {"precision": prec, "recall": rec, "f1": f1, "cssr": pairs.size / float(n_rows) ** 2,
            "identified": int(pairs.size), "true_pairs": int(truth.size), "true_identified": hit}

"""Shared by the GPU tests: the cost-model training recipe (logs of the
small person workload and a 100k-tuple draw of the plain recipe, trained by
the library's own kernels)."""
import numpy as np

from gen import workloads


def collect(hb, ctx, rel, rules, samples, seed):
    rid = hb.hb_load_relation(ctx, rel.columns, rel.n_rows)
    rs = hb.hb_compile_rules(ctx, rid, rules)
    hb.hb_partition(ctx, rid, rs)
    log = hb.hb_log_collect(ctx, rid, rs, samples, seed)
    hb.hb_release_relation(ctx, rid)
    return log


def train_model(hb, ctx):
    xs, ts = [], []
    for rel, rules in (workloads.person_small(), workloads.plain_1m(n=100_000)):
        log = collect(hb, ctx, rel, rules, 4, 7)
        xs.append(log["features"])
        ts.append(log["labels"])
    x = np.concatenate(xs)
    t = np.concatenate(ts)
    perm = np.random.default_rng(0).permutation(len(x))
    hb.hb_costmodel_init(ctx, 3)
    return hb.hb_costmodel_train(ctx, x[perm], t[perm], epochs=40, batch=256, lr=2e-3)

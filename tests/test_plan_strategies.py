"""The ordering strategies the paper's EPG tests compare against (cheapest
first, most selective first, random predicate order, random rule order),
through the pure-host hb_plan_path: each is a valid evaluation order of the
same rules, with the property that names it.  CPU only; the GPU parity of
every strategy is in test_gpu_parity.py."""
import numpy as np
import pytest

import paper_2410_04349_amd as hb


def instance(seed):
    r = np.random.default_rng(seed)
    n_preds = int(r.integers(3, 9))
    sp = r.random(n_preds)
    cost = r.random(n_preds) + 0.05
    rules = [sorted(set(r.integers(0, n_preds, size=int(r.integers(1, 5))).tolist())) for _ in range(int(r.integers(1, 7)))]
    return sp, cost, rules


@pytest.mark.parametrize("seed", range(20))
def test_single_criterion_orders(seed):
    sp, cost, rules = instance(seed)
    for plan, key in (("cheapest", cost), ("selective", sp)):
        path = hb.hb_plan_path(plan, sp, cost, rules)
        assert sorted(r for r, _ in path) == list(range(len(rules)))
        for r, preds in path:
            assert sorted(preds) == sorted(set(rules[r]))
            # ascending key, ties by predicate id (the ranking's stable order)
            assert preds == sorted(preds, key=lambda p: (key[p], p)), (plan, r, preds)


@pytest.mark.parametrize("seed", range(20))
def test_random_orders_permute_the_heuristic(seed):
    sp, cost, rules = instance(seed)
    heur = hb.hb_plan_path("heuristic", sp, cost, rules)
    rp = hb.hb_plan_path("random_preds", sp, cost, rules)
    rr = hb.hb_plan_path("random_rules", sp, cost, rules)
    assert [r for r, _ in rp] == [r for r, _ in heur]
    for (_, a), (_, b) in zip(rp, heur):
        assert sorted(a) == sorted(b)
    assert sorted(r for r, _ in rr) == sorted(r for r, _ in heur)
    assert dict(rr) == dict(heur)
    # fixed seed: repeated calls give the same order
    assert hb.hb_plan_path("random_preds", sp, cost, rules) == rp
    assert hb.hb_plan_path("random_rules", sp, cost, rules) == rr


def test_random_orders_do_reorder():
    # over many instances the random strategies must differ from the heuristic somewhere
    diff_p = diff_r = 0
    for seed in range(100, 160):
        sp, cost, rules = instance(seed)
        heur = hb.hb_plan_path("heuristic", sp, cost, rules)
        diff_p += hb.hb_plan_path("random_preds", sp, cost, rules) != heur
        diff_r += hb.hb_plan_path("random_rules", sp, cost, rules) != heur
    assert diff_p > 10 and diff_r > 10


def test_learned_and_unknown_plans_rejected():
    sp, cost, rules = instance(1)
    for plan in ("learned", 99):
        with pytest.raises(hb.HbError) as e:
            hb.hb_plan_path(plan, sp, cost, rules)
        assert e.value.status == hb.HB_ERR_INVALID_ARG

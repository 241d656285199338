"""Pins of the MCTS oracle's search logic with synthetic evaluators: exhaustion of a small
language, the first batch spreading over untried actions, enumeration-argmin recovery
under a full budget, and UCT concentrating visits on the rewarding subtree."""
import itertools

import numpy as np

from oracle import mcts as T
from oracle.sample import key_make, key_modes


def _synthetic(feasible_keys, J_of):
    def ev(keys, refine):
        J = np.array([J_of(k) for k in keys], float)
        v = np.array([0.0 if k in feasible_keys else 1.0 for k in keys])
        return J, v
    return ev


def test_first_batch_visits_every_single_segment_once():
    b = T.first_batch(0, kcap=1, P=12, seed=3)
    assert sorted(b) == sorted(key_make([i]) for i in range(12))


def test_search_returns_the_best_evaluated_order_without_repeats():
    """Distinct evaluated orders within the budget, each in the language, and the returned
    plan is the argmin of the evaluated feasible orders (refinement with the same values);
    with UCT's exploitation (c = 0.8, rewards in [0, 1]) the search may stall on the best
    subtree before the budget, which ends it after a fixed number of fruitless batches."""
    space = [list(p) for K in (1, 2) for p in itertools.product(range(12), repeat=K)]
    rng = np.random.default_rng(0)
    Jtab = {key_make(m): float(rng.uniform(1, 2)) for m in space}
    feas = {k for k in Jtab if rng.random() < 0.3}
    bk, bJ, bv, keys, J, v, nb, tree = T.mcts_search(0, None, None, None, kcap=2, P=16, eval_budget=len(space),
                                                     seed=1, knots_per_segment=5, k_ref=1000,
                                                     evaluate=_synthetic(feas, Jtab.get))
    assert len(set(keys)) == len(keys) <= len(space) and set(keys) <= set(Jtab)
    best = min((Jtab[k], k) for k in keys if k in feas)
    assert (bJ, bk) == best
    # a budget below the language size is met exactly
    out = T.mcts_search(0, None, None, None, kcap=2, P=16, eval_budget=40, seed=1, knots_per_segment=5, k_ref=10,
                        evaluate=_synthetic(feas, Jtab.get))
    assert len(out[3]) == 40


def test_flip_orders_stay_in_the_language():
    from oracle import flip as F
    ev = lambda keys, refine: (np.ones(len(keys)), np.ones(len(keys)))
    out = T.mcts_search(1, None, None, None, kcap=3, P=32, eval_budget=300, seed=4, knots_per_segment=5, k_ref=4,
                        evaluate=ev)
    assert len(out[3]) == 300 and all(F.admissible(key_modes(k)) for k in out[3])


def test_uct_concentrates_on_the_rewarding_subtree():
    # only orders starting with id 7 are feasible, the best is (7, 3)
    space = [list(p) for K in (1, 2) for p in itertools.product(range(12), repeat=K)]
    feas = {key_make(m) for m in space if m[0] == 7}
    J_of = lambda k: 1.0 if key_modes(k) == [7, 3] else 2.0
    bk, bJ, bv, keys, J, v, nb, tree = T.mcts_search(0, None, None, None, kcap=2, P=8, eval_budget=80, seed=2,
                                                     knots_per_segment=5, k_ref=10, evaluate=_synthetic(feas, J_of))
    visits = {a: ch.N for a, ch in tree.root.children}
    assert max(visits, key=visits.get) == 7
    assert visits[7] > 2 * sorted(visits.values())[-2]
    assert key_modes(bk) == [7, 3] and bJ == 1.0

"""Pins of the oracle's greedy contact-mode expansion (Alg. 1, Sec. III-B)."""
import itertools
import os

import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _edit1(m, M, kcap):
    out = set()
    K = len(m)
    for i in range(K):
        for a in range(M):
            if a != m[i]:
                out.add(m[:i] + (a,) + m[i + 1:])
    if K > 1:
        for i in range(K):
            out.add(m[:i] + m[i + 1:])
    if K < kcap:
        for i in range(K + 1):
            for a in range(M):
                out.add(m[:i] + (a,) + m[i:])
    out.discard(m)
    return out


def _runs(m):
    return 1 + sum(1 for i in range(1, len(m)) if m[i] != m[i - 1])


@pytest.mark.parametrize("m", [(0,), (5,), (1, 1), (2, 7, 2), (3, 3, 3), (0, 1, 1, 4), (9, 9, 2, 2, 11, 0)])
def test_one_edit_neighbourhood_closed_form_and_brute_force(orc, m):
    """|N_1(m)| over the product language with M ids and cap K_cap:
    K(M-1) substitutions + runs(m) distinct deletions (K>1) + (K+1)(M-1)+1 distinct
    insertions (K<K_cap); the set equals a brute-force set of one-edit orders."""
    M, kcap = 12, 6
    K = len(m)
    nb = orc.neighbours(list(m), M, kcap, 1)
    closed = K * (M - 1) + (_runs(m) if K > 1 else 0) + (((K + 1) * (M - 1) + 1) if K < kcap else 0)
    assert len(nb) == closed == len(set(nb))
    assert {tuple(orc.key_modes(k)) for k in nb} == _edit1(m, M, kcap)


@pytest.mark.parametrize("m", [(0,), (2, 7), (3, 3, 1)])
def test_two_edit_neighbourhood_is_bfs_over_admissible_orders(orc, m):
    """N_2(m): orders reachable by at most two edits with every intermediate admissible;
    the one-edit list comes first, then each neighbour's list, first occurrence kept."""
    M, kcap = 12, 3
    nb = orc.neighbours(list(m), M, kcap, 2)
    n1 = orc.neighbours(list(m), M, kcap, 1)
    assert nb[:len(n1)] == n1
    level1 = _edit1(m, M, kcap)
    both = set(level1)
    for q in level1:
        both |= _edit1(q, M, kcap)
    both.discard(m)
    assert len(nb) == len(set(nb))
    assert {tuple(orc.key_modes(k)) for k in nb} == both


def test_neighbourhood_enumeration_order_fixture(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "neighbourhood_order_push_M3.txt")) if l.strip()
            and not l.startswith("#")]
    expect = [[int(t) for t in r] for r in rows]
    got = [orc.key_modes(k) for k in orc.neighbours([0], 3, 2, 1)]
    assert got == expect


def test_key_order_is_segment_count_then_lexicographic(orc):
    seqs = [(0,), (11,), (0, 0), (0, 11), (1, 0), (0, 0, 0), (11, 11, 11, 11, 11, 11)]
    keys = [orc.key_make(s) for s in seqs]
    assert keys == sorted(keys)
    assert all(orc.key_modes(k) == list(s) for k, s in zip(keys, seqs))


def _tiny_expand(**kw):
    import oracle
    base = dict(kcap=2, seed_max_segments=1, radius=1, rounds=4, frontier_W=4096, knots_per_segment=5,
                k_ref=8, n_total=10, batch_B=100000, eval_budget=100000, mu_merit=100.0)
    base.update(kw)
    return oracle.Expand(**base)


@pytest.mark.parametrize("pair", [0, 1, 2])
def test_expansion_with_full_budget_equals_full_enumeration(orc, pair):
    """With a budget that covers the whole language, expansion evaluates every order and
    its refined argmin equals that of full enumeration followed by the same refinement
    (Sec. IV-A: full enumeration = every admissible order, same refinement)."""
    x0, goal, inst = I.push_pairs(0, 3)
    ep = _tiny_expand()
    r = orc.expand(x0[pair], goal[pair], inst[pair, 0], ep, eval_cap=1000)
    e = orc.enumerate_all(x0[pair], goal[pair], inst[pair, 0], ep)
    assert r["evaluated"] == e["evaluated"] == 12 + 144
    assert r["best_key"] == e["best_key"]
    if r["best_key"]:
        assert r["best_cost"] == e["best_cost"]


def test_expansion_batches_follow_algorithm_1(orc):
    """Seed = every order with at most s segments in key order; later batches hold only
    unseen orders, each a one-edit neighbour of an already evaluated order; no order is
    evaluated twice; batches never exceed B; rounds <= s_max + 1."""
    x0, goal, inst = I.push_pairs(5, 1)
    ep = _tiny_expand(kcap=3, seed_max_segments=1, rounds=2, batch_B=200, eval_budget=10000)
    r = orc.expand(x0[0], goal[0], inst[0, 0], ep, eval_cap=10000)
    keys = r["eval_keys"]
    assert keys[:12] == sorted(keys[:12]) and all(len(orc.key_modes(k)) == 1 for k in keys[:12])
    assert len(keys) == len(set(keys)) == r["evaluated"] <= 12 + 2 * 200
    nbs = {k: set(orc.neighbours(orc.key_modes(k), 12, 3, 1)) for k in keys}
    for i in range(12, len(keys)):
        assert any(keys[i] in nbs[p] for p in keys[:i])
    assert r["rounds"] <= ep.rounds + 1


def test_expansion_respects_evaluation_budget(orc):
    x0, goal, inst = I.push_pairs(6, 1)
    ep = _tiny_expand(kcap=3, rounds=5, batch_B=64, eval_budget=150)
    r = orc.expand(x0[0], goal[0], inst[0, 0], ep, eval_cap=1000)
    assert r["evaluated"] == 150

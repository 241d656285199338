"""The learned proposal inside the device expansion: it changes the order in which
candidate orders are solved, never which plan is returned.  A network trained on
evaluator results ranks each batch (queue order) and, optionally, seeds warm starts;
refinement re-solves the best feasible orders from the plain schedule-derived start in
both planners.  Warm-started solves begin with the tight penalty mu0_warm, so a good warm
start shortens every solve.  Asserted: identical returned plans, the first feasible order
comes earlier in evaluation order, and the device time to the first feasible plan is
shorter with the learned network than without it."""
import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu


def test_learned_expansion_returns_the_plain_plan_and_ranks_feasible_orders_first():
    import torch
    from paper_2609_21803_amd import learned, native
    data = learned.generate(262144, seed=4000)
    mlp = native.MLP(max_batch=16384, seed=1)
    log = learned.train(mlp, data, steps=800, batch=8192, lr=1e-3, log_every=200)
    print("training loss", log)
    assert log[-1][1][0] < log[0][1][0]
    ctx = native.Context(max_batch=16384, max_segments=6, max_intervals=24)
    prm = native.ExpandParams(kcap=3, seed_max_segments=2, radius=1, rounds=2, frontier_W=4096,
                              knots_per_segment=8, k_ref=64, batch_B=16384, eval_budget=20000, learned_warm=1)
    x0, goal, inst = I.push_pairs(9100, 8)          # held out: the training seeds are 4000+
    rows = learned.compare(ctx, mlp, prm, list(zip(x0, goal, inst)))
    same, ratios, first = 0, [], []
    for r in rows:
        p, l = r["plain"], r["learned"]
        print(p, l)
        assert p["evaluated"] == l["evaluated"]            # no batch truncation: same orders evaluated
        if p["modes"] == l["modes"] and (not p["modes"] or abs(p["cost"] - l["cost"]) <= 1e-4 * abs(p["cost"])):
            same += 1
        if p["t_first_ms"] > 0 and l["t_first_ms"] > 0:
            ratios.append(l["t_first_ms"] / p["t_first_ms"])
            first.append((p["first_index"], l["first_index"]))
    print("TTFP ratios learned/plain", ratios, "first feasible index (plain, learned)", first)
    assert same >= 7
    first = np.array(first)
    assert len(first) >= 4 and np.median(first[:, 1]) < np.median(first[:, 0])
    assert len(ratios) >= 4 and np.median(ratios) < 0.9

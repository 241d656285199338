"""GPU parity of the flipping evaluator against the FP64 flip oracle (same inputs, same
algorithm).  Both sides compute in FP64; differences come from summation order and the
device's sin/cos, so iterates agree closely until a near-tie discrete decision (an
accepted vs rejected trial step, an active-set change) separates them.  Sequence by
sequence, the rule of tests/parity.py holds: identical flags on every margin sequence and
the objective within 1e-4 where both are feasible, a disagreement excused only where the
flip oracle itself changes its answer under one-ulp input moves (each one printed)."""
import numpy as np
import pytest

import parity
from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu

fid = lambda f1, f2, g: (f1 * 13 + f2) * 5 + g
fg = lambda face, slip: 1 + 3 * face + slip


def _pivot_px(th):
    c = np.array([-0.1, -0.05])
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    return -0.1 - (R @ c)[0]


def designed_batch():
    """orders with kinematically consistent goals (pivot about the bottom-left corner),
    slides and rests, on several table frictions"""
    rows = []
    for th in (0.9, 1.2, 1.45):
        for mu in (0.62, 0.7, 0.78):
            rows.append(([fid(fg(0, 1), 0, 0), fid(fg(0, 0), 0, 3)], [10, 10], (_pivot_px(th), th), mu))
            rows.append(([fid(0, 0, 0), fid(fg(0, 0), fg(1, 0), 3)], [10, 10], (_pivot_px(th), th), mu))
    for d in (0.02, 0.05, -0.04):
        rows.append(([fid(fg(2 if d > 0 else 0, 0), 0, 1 if d > 0 else 2)], [8], (d, 0.0), 0.7))
    rows.append(([fid(0, 0, 0), fid(fg(0, 0), 0, 0)], [4, 4], (0.0, 0.0), 0.7))
    B = len(rows)
    b = dict(x0=np.tile(np.array(I.FLIP_X0), (B, 1)), goal=np.array([r[2] for r in rows]),
             inst=np.array([[r[3]] for r in rows]), nseg=np.array([len(r[0]) for r in rows], np.int32),
             modes=np.zeros((B, 6), np.int32), knots=np.zeros((B, 6), np.int32))
    for i, r in enumerate(rows):
        b["modes"][i, :len(r[0])] = r[0]
        b["knots"][i, :len(r[1])] = r[1]
    return b


def _run(ctx, b, **kw):
    import torch
    from paper_2609_21803_amd import native
    d = native.to_device(b)
    out = ctx.evaluate(**d, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _oracle(b, **kw):
    from oracle import flip as F
    return F.evaluate(_f32(b["x0"]), _f32(b["goal"]), _f32(b["inst"]), b["nseg"], b["modes"], b["knots"], **kw)


def _parity(g, o, b, label, idx=None, warm=None, **kw):
    def solve(sub, rows, r32):   # the flipping evaluator is FP64 throughout: input draws only
        return _oracle(sub, warm=None if warm is None else warm[rows], **kw)
    return parity.check(g, o, b, solve, label, idx=idx)


def test_designed_flips_match_oracle():
    from paper_2609_21803_amd import native
    b = designed_batch()
    ctx = native.Context(max_batch=256, max_intervals=60, task=native.TASK_FLIP)
    g = _run(ctx, b)
    o = _oracle(b)
    print("feasible gpu", g["feasible"].sum(), "oracle", o["feasible"].sum(), "of", len(g["feasible"]))
    assert o["feasible"].sum() >= 10
    assert np.array_equal(g["feasible"], o["feasible"])
    both = (g["feasible"] == 1) & (o["feasible"] == 1)
    rel = np.abs(g["cost"] - o["cost"]) / np.maximum(np.abs(o["cost"]), 1e-12)
    assert (rel[both] <= 1e-4).all(), rel[both]
    assert (g["viol"][both] <= 1e-5).all()
    assert np.array_equal(g["stats"][:, 3], o["stats"][:, 3])


def test_random_orders_match_oracle():
    """Random (mostly infeasible) orders solved to the end of the budget: same status and,
    on most orders, the same final cost and violation."""
    from paper_2609_21803_amd import native
    b = I.flip_tiny()
    ctx = native.Context(max_batch=1024, max_intervals=15, task=native.TASK_FLIP)
    g = _run(ctx, b)
    o = _oracle(b)
    scale = np.maximum(np.abs(o["cost"]), 1e-3)
    close = (np.abs(g["cost"] - o["cost"]) <= 1e-4 * scale) & (np.abs(g["viol"] - o["viol"]) <= 1e-5 + 1e-4 * o["viol"])
    same_it = (g["stats"][:, :2] == o["stats"][:, :2]).all(1)
    print("close", close.mean(), "same iteration counts", same_it.mean(), "feasible", g["feasible"].sum(),
          o["feasible"].sum())
    _parity(g, o, b, "flip random orders")
    assert close.mean() >= 0.9
    assert (g["stats"][:, 3] == o["stats"][:, 3]).mean() >= 0.95


def test_warm_start_matches_oracle_with_same_warm_start():
    from paper_2609_21803_amd import native
    import torch
    b = designed_batch()
    o = _oracle(b, nmax=60)
    warm = o["traj"].astype(np.float32)
    ctx = native.Context(max_batch=256, max_intervals=60, task=native.TASK_FLIP)
    g = _run(ctx, b, warm=torch.as_tensor(warm).cuda())
    ow = _oracle(b, warm=warm.astype(np.float64), nmax=60)
    assert np.array_equal(g["feasible"], ow["feasible"])
    both = (g["feasible"] == 1) & (ow["feasible"] == 1)
    rel = np.abs(g["cost"] - ow["cost"]) / np.maximum(np.abs(ow["cost"]), 1e-12)
    assert (rel[both] <= 1e-4).all()


def test_invalid_orders_flagged_and_batch_independent():
    from paper_2609_21803_amd import native
    b = I.flip_tiny(B=64)
    b["modes"][3, 0] = 845                                     # out of range id
    b["nseg"][5], b["modes"][5, :2], b["knots"][5, :2] = 2, (fid(fg(0, 0), 0, 3), fid(fg(1, 0), 0, 4)), 5
    ctx = native.Context(max_batch=128, max_intervals=15, task=native.TASK_FLIP)
    g = _run(ctx, b)
    assert np.isnan(g["cost"][3]) and np.isinf(g["viol"][3]) and g["stats"][3, 3] == 3
    assert np.isnan(g["cost"][5]) and g["stats"][5, 3] == 3
    with pytest.raises(native.CometError):
        ctx.check()
    ctx.check()                                                # the counter was cleared
    # the same orders in another batch composition give bit-identical results
    idx = np.array([10, 2, 40, 7])
    g2 = _run(ctx, I.subset(b, idx))
    for k in ("cost", "viol", "feasible", "stats"):
        assert np.array_equal(g2[k], g[k][idx], equal_nan=True), k


def test_full_size_flip_workload_sampled():
    """The benchmark's flipping round (32,768 orders, K ~ U{1..6}, 10 intervals per
    segment, up to 60 intervals) in the launch configuration bench.py times: 512 evenly
    strided orders re-solved by the oracle agree; prints solves/s."""
    from paper_2609_21803_amd import native
    import torch
    b = I.flip_batch(3100, 32768)
    ctx = native.Context(max_batch=32768, max_intervals=60, task=native.TASK_FLIP)
    d = native.to_device(b)
    out = ctx.evaluate(**d)
    torch.cuda.synchronize()
    ms = ctx.kernel_ms()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    print(f"flip 32768 orders: {ms:.1f} ms, {32768 / ms * 1e3:.0f} solves/s, mean GN {g['stats'][:, 1].mean():.1f}")
    idx = np.linspace(0, 32767, 512).astype(np.int64)
    o = _oracle(I.subset(b, idx), nmax=60)
    scale = np.maximum(np.abs(o["cost"]), 1e-3)
    close = (np.abs(g["cost"][idx] - o["cost"]) <= 1e-4 * scale) & \
            (np.abs(g["viol"][idx] - o["viol"]) <= 1e-5 + 1e-4 * o["viol"])
    print("sampled close", close.mean())
    _parity({k: g[k][idx] for k in ("cost", "viol", "feasible")}, o, I.subset(b, idx), "flip 32,768 (strided)",
            idx=idx, nmax=60)
    assert close.mean() >= 0.9
    assert (g["stats"][idx, 3] == o["stats"][:, 3]).mean() >= 0.95
    assert np.array_equal(g["traj"][idx, :, :].shape, (512, 61, 17))


def test_empty_batch_and_oversized_orders():
    from paper_2609_21803_amd import native
    ctx = native.Context(max_batch=16, max_intervals=10, task=native.TASK_FLIP)
    b = I.flip_tiny(B=4)
    b["knots"][1, :] = 0
    b["nseg"][1], b["knots"][1, :3] = 3, (5, 5, 5)               # 15 intervals > max_intervals
    # a knot count whose int32 sum with the earlier ones would wrap negative
    b["knots"][2, :] = 0
    b["nseg"][2], b["knots"][2, :2] = 2, (5, 2 ** 31 - 1)
    g = _run(ctx, b)
    for i in (1, 2):
        assert np.isnan(g["cost"][i]) and g["stats"][i, 3] == 3
    with pytest.raises(native.CometError):
        ctx.check()
    import torch
    e = {k: v[:0] for k, v in native.to_device(b).items()}
    ctx.evaluate(**e)                                             # B = 0 is a no-op
    torch.cuda.synchronize()


def test_maximum_length_orders_match_oracle():
    """Six segments x 85 intervals = 510 of the 512 intervals a context holds (the work
    space's largest per-order extent): same status as the oracle on every order, the same
    final cost and violation on most (solved to the end of the budget), rows beyond N zero."""
    from paper_2609_21803_amd import native
    b = I.flip_batch(5100, 8, n_pairs=4, kmin=6, kmax=6, knots=85)
    ctx = native.Context(max_batch=8, max_intervals=512, task=native.TASK_FLIP)
    g = _run(ctx, b)
    ctx.check()
    o = _oracle(b, nmax=512)
    scale = np.maximum(np.abs(o["cost"]), 1e-3)
    close = (np.abs(g["cost"] - o["cost"]) <= 1e-4 * scale) & (np.abs(g["viol"] - o["viol"]) <= 1e-5 + 1e-4 * o["viol"])
    print("maximum length: close", close.tolist(), "status", g["stats"][:, 3].tolist(), o["stats"][:, 3].tolist())
    assert np.array_equal(g["feasible"], o["feasible"]) and np.array_equal(g["stats"][:, 3], o["stats"][:, 3])
    assert close.sum() >= 6
    assert np.all(g["traj"][:, 511:] == 0)

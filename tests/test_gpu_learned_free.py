"""The learned proposal for pushing with free motion (eight segment slots, 16 ids), with the
fixed step and with optimised timing.

* Encoding, targets and warm-start decode against the oracle on evaluator results of
  admissible orders of up to eight segments with ragged interval counts: the encoding bit
  for bit up to one BF16 step on the trigonometric entries, the targets and masks to
  float32 interpolation, the decode of the targets as network outputs to float32.
* A network trained on the evaluator's results of uniformly sampled orders, inside the
  device expansion: ranking alone leaves the evaluated set and the returned plan exactly
  the plain planner's (the queue order never changes a result) and moves the first
  feasible order forward in the queue; with warm starts the returned plan, re-solved from
  the plain start, is never worse than the plain planner's with the fixed step, and within
  a few per cent of it with optimised timing.
"""
import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu


def _orders(rng, B, kmax=8):
    from oracle import free as F
    keys = F.seed(kmax)
    pick = rng.choice(len(keys), B, replace=False)
    nseg = np.zeros(B, np.int32)
    modes = np.zeros((B, 8), np.int32)
    knots = np.zeros((B, 8), np.int32)
    for i, p in enumerate(pick):
        m = F.key_modes(int(keys[p]))
        nseg[i] = len(m)
        modes[i, :len(m)] = m
        knots[i, :len(m)] = rng.integers(1, 11, len(m))
    return nseg, modes, knots


@pytest.mark.parametrize("timed", [False, True])
def test_free_encode_targets_and_decode_match_oracle(timed):
    import torch
    from oracle.mlp import bf16_bits, decode_warm_free, encode_free, targets
    from paper_2609_21803_amd import native
    task = native.TASK_PUSH_FREE_TIMED if timed else native.TASK_PUSH_FREE
    rng = np.random.default_rng(31 + timed)
    B, nmax = 512, 80
    nseg, modes, knots = _orders(rng, B)
    x0, goal, inst = I.push_free_pairs(7000 + timed, 16)
    pair = rng.integers(0, 16, B)
    b = dict(x0=x0[pair], goal=goal[pair], inst=inst[pair], nseg=nseg, modes=modes, knots=knots)
    d = native.to_device(b)
    in_dim, out_dim = native.mlp_dims(task)
    assert (in_dim, out_dim) == (528, 968)
    x = native.mlp_encode(d, task=task).cpu().numpy().view(np.uint16)
    ref = bf16_bits(encode_free(b["x0"], b["goal"], b["inst"], nseg, modes, knots))
    diff = x.astype(np.int32) - ref.astype(np.int32)
    assert np.all(np.abs(diff) <= 1)
    assert np.all(diff[:, [0, 1, 4, 5, 8, 9, 10, 11, 12, 13]] == 0) and np.all(diff[:, 16:] == 0)

    ctx = native.Context(max_batch=B, max_segments=8, max_intervals=nmax, task=task)
    out = ctx.evaluate(**d)
    torch.cuda.synchronize()
    yf, yc, yt, mk = [a.cpu().numpy() for a in native.mlp_targets(d, out, nmax, task=task)]
    assert yt.shape == (B, 960)
    tr = out["traj"].cpu().numpy().astype(np.float64)
    fe = out["feasible"].cpu().numpy()
    co = out["cost"].cpu().numpy().astype(np.float64)
    cols = [0, 1, 2, 3, 4, 5, 6] + ([9] if timed else [])
    ryf, ryc, ryt, rmk = targets(tr, nseg, knots, fe, co, nch=len(cols), n_seg=8, cols=cols)
    assert np.array_equal(yf, ryf) and np.array_equal(mk, rmk)
    assert np.allclose(yc, ryc, atol=1e-6)
    scale = np.abs(tr).reshape(B, -1).max(axis=1, keepdims=True)
    assert np.all(np.abs(yt - ryt) <= 1e-5 + 1e-6 * scale)      # float32 interpolation
    print("feasible orders", int(fe.sum()), "of", B)

    # the targets decoded as network outputs; the oracle decodes the same float32 values
    Y = torch.zeros((B, out_dim), device="cuda")
    Y[:, 2:962] = torch.as_tensor(yt).cuda()
    w = native.mlp_decode_warm(Y, d, nmax, task=task).cpu().numpy()
    rw = decode_warm_free(Y.cpu().numpy().astype(np.float64), b["x0"].astype(np.float32).astype(np.float64), nseg,
                          knots, nmax, timed=timed)
    assert w.shape == rw.shape == (B, nmax + 1, 10 if timed else 9)
    # states, forces and durations: float32 interpolation; velocities: a difference of two
    # decoded positions over the duration, so the bound scales with position / h
    pos = np.abs(rw[:, :, :7]).max(axis=(1, 2))[:, None, None]
    assert np.all(np.abs(w[:, :, :7] - rw[:, :, :7]) <= 1e-5 + 1e-6 * pos)
    if timed:
        assert np.allclose(w[:, :, 9], rw[:, :, 9], atol=1e-6)
    h = rw[:, :, 9:10] if timed else 0.1
    assert np.all(np.abs(w[:, :, 7:9] - rw[:, :, 7:9]) <= (2e-5 + 2e-6 * pos) / np.maximum(h, 0.02) + 1e-5)


def _free_rows(mlp, warm, task):
    from paper_2609_21803_amd import learned, native
    ctx = native.Context(max_batch=16384, max_segments=8, max_intervals=24, task=task)
    prm = native.ExpandParams(kcap=6, seed_max_segments=2, radius=2, rounds=2, frontier_W=1024, knots_per_segment=0,
                              n_total=24, k_ref=64, batch_B=16384, eval_budget=40000, learned_warm=warm)
    x0, goal, inst = I.push_free_pairs(9300, 8)     # held out: the training seeds are 6000+
    return learned.compare(ctx, mlp, prm, list(zip(x0, goal, inst)))


@pytest.mark.parametrize("timed", [False, True])
def test_free_learned_ranking_keeps_the_plain_plan_and_warm_starts_do_not_lose(timed):
    """Ranking alone: the plain planner's evaluated set, feasible count, order and cost on
    every goal, and an earlier first feasible order.  With warm starts: with the fixed step
    a plan no worse than the plain one (1e-4 relative) on every goal; with optimised timing,
    where a warm start can settle a solve in another local optimum of the durations (as for
    timed pushing), within 3 % of the plain plan's cost on every goal."""
    from paper_2609_21803_amd import learned, native
    task = native.TASK_PUSH_FREE_TIMED if timed else native.TASK_PUSH_FREE
    gen = native.Context(max_batch=16384, max_segments=8, max_intervals=24, task=task)
    data = learned.generate_free(16, 16384, seed=6000, ctx=gen, kcap=6, n_total=24)
    feas = float(data["y_feas"].mean())
    in_dim, out_dim = native.mlp_dims(task)
    mlp = native.MLP(max_batch=16384, seed=1, in_dim=in_dim, out_dim=out_dim)
    log = learned.train(mlp, data, steps=800, batch=8192, lr=1e-3, log_every=200)
    print("free training: samples", int(data["X"].shape[0]), "feasible fraction", feas, "loss", log)
    assert log[-1][1][0] < log[0][1][0]

    rows = _free_rows(mlp, 0, task)
    first = []
    for r in rows:
        p, l = r["plain"], r["learned"]
        print(p, l)
        assert p["evaluated"] == l["evaluated"] and p["n_feasible"] == l["n_feasible"]
        assert p["modes"] == l["modes"]
        assert (not p["modes"]) or abs(p["cost"] - l["cost"]) <= 1e-4 * abs(p["cost"])
        if p["t_first_ms"] > 0 and l["t_first_ms"] > 0:
            first.append((p["first_index"], l["first_index"]))
    print("ranking only: first feasible index (plain, learned)", first)
    first = np.array(first)
    assert len(first) >= 4 and np.median(first[:, 1]) < np.median(first[:, 0])

    rows = _free_rows(mlp, 1, task)
    rel, ratios = [], []
    for r in rows:
        p, l = r["plain"], r["learned"]
        print("warm", p, l)
        if p["modes"]:
            assert l["modes"]
            rel.append((l["cost"] - p["cost"]) / p["cost"])
        if p["t_first_ms"] > 0 and l["t_first_ms"] > 0:
            ratios.append(l["t_first_ms"] / p["t_first_ms"])
    print("warm starts: returned cost learned/plain - 1", rel, "TTFP ratios learned/plain", ratios)
    assert len(rel) >= 4
    if timed:
        assert max(abs(x) for x in rel) <= 0.03
    else:
        assert max(rel) <= 1e-4

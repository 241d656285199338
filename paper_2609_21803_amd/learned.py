"""Training data, training loop and plain-vs-learned comparison for the proposal network.

Every numerical step runs in the HIP library (evaluator, target builder, encoder, BF16
matrix-core training kernels); this module only draws seeded batches, slices device
buffers into minibatches and loops.
"""
from __future__ import annotations

import math

import numpy as np

from . import instances as I
from . import native


def generate(n_samples: int, seed: int = 4000, chunk: int = 65536, kmin=1, kmax=5, nmin=5, nmax=15,
             ctx: native.Context | None = None):
    """Evaluate n_samples seeded ragged pushing orders and build (X, targets) on the GPU
    (fixed-step pushing, or optimised timing when `ctx` is a timed context)."""
    import torch
    N = 6 * nmax
    ctx = ctx or native.Context(max_batch=chunk, max_segments=6, max_intervals=N)
    X = torch.empty((n_samples, native.MLP.IN), dtype=torch.int16, device="cuda")
    yf = torch.empty(n_samples, device="cuda")
    yc = torch.empty(n_samples, device="cuda")
    yt = torch.empty((n_samples, 720), device="cuda")
    mk = torch.empty((n_samples, 720), device="cuda")
    done, i = 0, 0
    while done < n_samples:
        B = min(chunk, n_samples - done)
        b = I.push_hetero(seed=seed + i, B=B, kmin=kmin, kmax=kmax, nmin=nmin, nmax=nmax)
        d = native.to_device(b)
        out = ctx.evaluate(**d)
        X[done:done + B] = native.mlp_encode(d, task=ctx.task)
        f, c, t, m = native.mlp_targets(d, out, ctx.max_intervals, task=ctx.task)
        yf[done:done + B], yc[done:done + B], yt[done:done + B], mk[done:done + B] = f, c, t, m
        done += B
        i += 1
    return dict(X=X, y_feas=yf, y_cost=yc, y_traj=yt, mask=mk)


def flip_seed_keys(ctx: native.Context, kcap: int = 2, knots: int = 10):
    """The filtered single-segment seed of the flipping expansion (Alg. 1's first
    frontier), read back from a zero-round device expansion."""
    import torch
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    x0, goal, inst = I.flip_pairs(1, 1)
    prm = native.ExpandParams(kcap=kcap, seed_max_segments=1, radius=1, rounds=0, frontier_W=1,
                              knots_per_segment=knots, k_ref=0, batch_B=min(ctx.max_batch, 4096), eval_budget=4096)
    native.expand(ctx, t(x0[0]), t(goal[0]), t(inst[0]), prm)
    keys, _, _ = native.expand_trace(ctx)
    return keys.clone()


def decode_keys(keys, smax: int = 6, bits: int = 10):
    """Order keys (the segment count at bit 60, then `bits` bits per mode id from bit
    60 - bits down: 10 for pushing, timed pushing and flipping, 4 for free motion) ->
    nseg, modes."""
    import torch
    nseg = ((keys >> 60) & 15).to(torch.int32)    # keys arrive as int64: K = 8 sets the sign bit
    shifts = torch.tensor([60 - bits * (j + 1) for j in range(smax)], device=keys.device, dtype=torch.int64)
    modes = ((keys[:, None] >> shifts[None, :]) & ((1 << bits) - 1)).to(torch.int32)
    modes = torch.where(torch.arange(smax, device=keys.device)[None, :] < nseg[:, None], modes, 0)
    return nseg, modes


def split_knots(nseg, smax: int, n_total: int):
    """n_total intervals per order split evenly over its segments, one more for each of the
    first n_total mod K (the expansion's allocation when knots_per_segment is 0)."""
    import torch
    j = torch.arange(smax, device=nseg.device)[None, :]
    K = nseg.clamp(min=1)[:, None]
    return torch.where(j < nseg[:, None], n_total // K + (j < n_total % K).to(K.dtype), 0).to(torch.int32)


def generate_free(n_instances: int, per_instance: int, seed: int = 6000, ctx: native.Context | None = None,
                  kcap: int = 8, n_total: int = 50, chunk: int = 16384):
    """Free-motion training data: on each seeded start/goal pair (``push_free_pairs``),
    `per_instance` distinct admissible orders of up to kcap segments drawn by the device's
    uniform sampler (each segment count equally likely, then every admissible order of
    that count), n_total intervals per order split evenly; every order is solved by the
    evaluator and turned into (X, targets) on the GPU.  `ctx` fixes the task (free motion
    with the fixed step or with optimised timing)."""
    import torch
    ctx = ctx or native.Context(max_batch=chunk, max_segments=8, max_intervals=n_total, task=native.TASK_PUSH_FREE)
    task = ctx.task
    B = min(chunk, ctx.max_batch, per_instance)
    prm = native.ExpandParams(kcap=kcap, seed_max_segments=1, radius=1, rounds=(per_instance + B - 1) // B + 8,
                              frontier_W=1, knots_per_segment=0, n_total=n_total, k_ref=0, batch_B=B,
                              eval_budget=per_instance, policy=native.POLICY_UNIFORM, sample_draws=4 * B)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    x0, goal, inst = I.push_free_pairs(seed, n_instances)
    in_dim, _ = native.mlp_dims(task)
    W = 120 * native.mlp_segments(task)
    parts = []
    for i in range(n_instances):
        prm.sample_seed = seed * 1000 + i
        native.expand(ctx, f32(x0[i]), f32(goal[i]), f32(inst[i]), prm)
        keys = native.expand_trace(ctx)[0].clone()
        nseg, modes = decode_keys(keys, smax=ctx.max_segments, bits=4)
        kn = split_knots(nseg, ctx.max_segments, n_total)
        n = int(keys.shape[0])
        X = torch.empty((n, in_dim), dtype=torch.int16, device="cuda")
        yf, yc = torch.empty(n, device="cuda"), torch.empty(n, device="cuda")
        yt, mk = torch.empty((n, W), device="cuda"), torch.empty((n, W), device="cuda")
        for s in range(0, n, ctx.max_batch):
            e = min(n, s + ctx.max_batch)
            d = dict(x0=f32(x0[i])[None].expand(e - s, -1).contiguous(),
                     goal=f32(goal[i])[None].expand(e - s, -1).contiguous(),
                     inst=f32(inst[i]).reshape(1, 1).expand(e - s, 1).contiguous(), nseg=nseg[s:e].contiguous(),
                     modes=modes[s:e].contiguous(), knots=kn[s:e].contiguous())
            out = ctx.evaluate(**d)
            X[s:e] = native.mlp_encode(d, task=task)
            yf[s:e], yc[s:e], yt[s:e], mk[s:e] = native.mlp_targets(d, out, ctx.max_intervals, task=task)
        ctx.check()                      # every sampled order must have been a valid one
        parts.append((X, yf, yc, yt, mk))
    cat = lambda k: torch.cat([p[k] for p in parts])
    return dict(X=cat(0), y_feas=cat(1), y_cost=cat(2), y_traj=cat(3), mask=cat(4))


def generate_flip(n_instances: int, seed: int = 5000, ctx: native.Context | None = None, kcap: int = 2,
                  parents: int = 16, room: int = 1024, knots: int = 10, chunk: int = 32768, pairs=I.flip_pivot_pairs):
    """Flipping training data: on each seeded start/goal pair (``pairs(seed, n)``), the
    expansion's seed orders plus `room` neighbours (one edit) of `parents` random seed
    orders, built by the device batch constructor; every order is solved by the evaluator
    and turned into (X, targets) on the GPU."""
    import torch
    ctx = ctx or native.Context(max_batch=chunk, max_segments=6, max_intervals=kcap * knots, task=native.TASK_FLIP)
    seed_keys = flip_seed_keys(ctx, kcap, knots)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    prm = native.ExpandParams(kcap=kcap, seed_max_segments=1, radius=1, rounds=1, frontier_W=parents,
                              knots_per_segment=knots, k_ref=0, batch_B=room, eval_budget=room)
    x0, goal, inst = pairs(seed, n_instances)
    keys, pair = [], []
    for i in range(n_instances):
        merit = torch.rand(seed_keys.shape[0], generator=g, device="cuda", dtype=torch.float64)
        nb = native.expand_next(ctx, seed_keys, merit, prm, room)
        keys.append(torch.cat([seed_keys, nb]))
        pair.append(torch.full((keys[-1].shape[0],), i, dtype=torch.int64, device="cuda"))
    keys, pair = torch.cat(keys), torch.cat(pair)
    n = int(keys.shape[0])
    nseg, modes = decode_keys(keys)
    kn = torch.where(modes.new_ones(modes.shape).cumsum(1) <= nseg[:, None], knots, 0).to(torch.int32)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    X0, G, M = f32(x0)[pair], f32(goal)[pair], f32(inst)[pair]
    X = torch.empty((n, native.MLP.IN), dtype=torch.int16, device="cuda")
    yf = torch.empty(n, device="cuda")
    yc = torch.empty(n, device="cuda")
    yt = torch.empty((n, 720), device="cuda")
    mk = torch.empty((n, 720), device="cuda")
    for s in range(0, n, ctx.max_batch):
        e = min(n, s + ctx.max_batch)
        d = dict(x0=X0[s:e].contiguous(), goal=G[s:e].contiguous(), inst=M[s:e].contiguous(),
                 nseg=nseg[s:e].contiguous(), modes=modes[s:e].contiguous(), knots=kn[s:e].contiguous())
        out = ctx.evaluate(**d)
        X[s:e] = native.mlp_encode(d, task=native.TASK_FLIP)
        f, c, t, m = native.mlp_targets(d, out, ctx.max_intervals, task=native.TASK_FLIP)
        yf[s:e], yc[s:e], yt[s:e], mk[s:e] = f, c, t, m
    return dict(X=X, y_feas=yf, y_cost=yc, y_traj=yt, mask=mk)


def train(mlp: native.MLP, data: dict, steps: int, batch: int = 8192, lr: float = 1e-3, seed: int = 0,
          weight_decay: float = 1e-4, log_every: int = 0):
    """AdamW with cosine learning-rate decay over random minibatches; returns the loss log."""
    import torch
    n = data["X"].shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    log = []
    for s in range(steps):
        idx = torch.randint(0, n, (batch,), device="cuda", generator=g)
        lr_s = lr * 0.5 * (1 + math.cos(math.pi * s / max(steps, 1)))
        loss = mlp.train_step(data["X"].index_select(0, idx).contiguous(), data["y_feas"].index_select(0, idx),
                              data["y_cost"].index_select(0, idx), data["y_traj"].index_select(0, idx).contiguous(),
                              data["mask"].index_select(0, idx).contiguous(), lr_s, weight_decay)
        if log_every and (s % log_every == 0 or s == steps - 1):
            log.append((s, loss.cpu().numpy().tolist()))
    return log


def compare(ctx: native.Context, mlp: native.MLP, params: native.ExpandParams, pairs, trace: bool = False):
    """Plain vs learned expansion on each (x0, goal, inst): time and evaluations to the first
    feasible plan, and the returned plan of each (with trace, also the plain expansion's
    evaluated keys and (J, v) in evaluation order)."""
    import torch
    rows = []
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    for x0, goal, inst in pairs:
        rec = {}
        for name, net in (("plain", None), ("learned", mlp)):
            o, st = native.expand(ctx, t(x0), t(goal), t(inst), params, learned=net)
            torch.cuda.synchronize()
            K = int(o["nseg"].item())
            rec[name] = dict(t_first_ms=st["t_first_feasible_ms"], first_index=st["first_feasible_index"],
                             t_total_ms=st["t_total_ms"], evaluated=st["evaluated"], n_feasible=st["n_feasible"],
                             cost=float(o["cost"].item()), modes=o["modes"].cpu().numpy()[:K].tolist())
            if trace and net is None:
                k, J, v = native.expand_trace(ctx)
                rec[name]["trace"] = (k.clone(), J.cpu().numpy(), v.cpu().numpy())
        rows.append(rec)
    return rows


def auc(score, label) -> float:
    """Area under the ROC curve of `score` for the binary `label` (Mann-Whitney, ties half)."""
    score = np.asarray(score, np.float64)
    label = np.asarray(label, bool)
    npos, nneg = int(label.sum()), int((~label).sum())
    if npos == 0 or nneg == 0:
        return float("nan")
    order = np.argsort(score, kind="mergesort")
    ranks = np.empty(len(score))
    s = score[order]
    i = 0
    while i < len(s):                      # average ranks over ties
        j = i
        while j + 1 < len(s) and s[j + 1] == s[i]:
            j += 1
        ranks[order[i:j + 1]] = 0.5 * (i + j) + 1.0
        i = j + 1
    return float((ranks[label].sum() - npos * (npos + 1) / 2) / (npos * nneg))


def feasibility_auc(mlp: native.MLP, keys, feasible, x0, goal, inst, knots_per_segment: int, task=native.TASK_PUSH,
                    n_total: int = 0):
    """AUC of the network's feasibility logit over evaluated orders (keys on the device) of one
    instance, against the evaluator's flags (knots_per_segment <= 0: n_total intervals split
    evenly, as the expansion allocates them)."""
    import torch
    n = int(keys.shape[0])
    S = native.mlp_segments(task)
    nseg, modes = decode_keys(keys, smax=S, bits=4 if S == 8 else 10)
    if knots_per_segment > 0:
        kn = torch.where(modes.new_ones(modes.shape).cumsum(1) <= nseg[:, None], knots_per_segment, 0).to(torch.int32)
    else:
        kn = split_knots(nseg, S, n_total)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    logits = []
    for s in range(0, n, mlp.max_batch):
        e = min(n, s + mlp.max_batch)
        d = dict(x0=f32(x0)[None].expand(e - s, -1).contiguous(), goal=f32(goal)[None].expand(e - s, -1).contiguous(),
                 inst=f32(inst).reshape(1, 1).expand(e - s, 1).contiguous(), nseg=nseg[s:e].contiguous(),
                 modes=modes[s:e].contiguous(), knots=kn[s:e].contiguous())
        logits.append(mlp.forward(native.mlp_encode(d, task=task))[:, 0].float().cpu().numpy())
    return auc(np.concatenate(logits), feasible)


def warm_start_savings(ctx: native.Context, mlp: native.MLP, batch: dict):
    """Gauss-Newton iterations of the plain schedule-derived start against the network's warm
    start on one batch: mean iterations over the orders feasible from both starts, and the
    feasible fractions."""
    import torch
    d = native.to_device(batch)
    plain = ctx.evaluate(**d)
    torch.cuda.synchronize()
    Y = torch.cat([mlp.forward(native.mlp_encode({k: v[s:s + mlp.max_batch] for k, v in d.items()}, task=ctx.task))
                   for s in range(0, int(d["nseg"].shape[0]), mlp.max_batch)])
    warm = native.mlp_decode_warm(Y, d, ctx.max_intervals, task=ctx.task)
    ws = ctx.evaluate(**d, warm=warm)
    torch.cuda.synchronize()
    fp, fw = plain["feasible"].cpu().numpy() == 1, ws["feasible"].cpu().numpy() == 1
    gp, gw = plain["stats"].cpu().numpy()[:, 1], ws["stats"].cpu().numpy()[:, 1]
    both = fp & fw
    return dict(orders=int(len(fp)), feasible_plain=float(fp.mean()), feasible_warm=float(fw.mean()),
                gn_plain_mean=float(gp[both].mean()), gn_warm_mean=float(gw[both].mean()),
                gn_saved_fraction=float(1.0 - gw[both].mean() / gp[both].mean()),
                gn_all_plain_mean=float(gp.mean()), gn_all_warm_mean=float(gw.mean()))

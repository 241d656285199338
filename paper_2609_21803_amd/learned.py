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
    """Evaluate n_samples seeded ragged pushing orders and build (X, targets) on the GPU."""
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
        X[done:done + B] = native.mlp_encode(d)
        f, c, t, m = native.mlp_targets(d, out, ctx.max_intervals)
        yf[done:done + B], yc[done:done + B], yt[done:done + B], mk[done:done + B] = f, c, t, m
        done += B
        i += 1
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


def compare(ctx: native.Context, mlp: native.MLP, params: native.ExpandParams, pairs):
    """Plain vs learned expansion on each (x0, goal, inst): time and evaluations to the first
    feasible plan, and the returned plan of each."""
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
        rows.append(rec)
    return rows

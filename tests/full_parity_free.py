"""The whole 118,080-order free-motion benchmark launch against the oracle, sequence by sequence
under the parity rule of tests/parity.py: every admissible order of at most six segments on 8
instances, with the fixed step (10 intervals per segment) or, with the argument `timed`, with
optimised timing (50 intervals per order, split evenly).  The oracle takes about 4.5 (7)
minutes on 16 threads, so this is a script, run by hand on a GPU machine:
python tests/full_parity_free.py [timed]."""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)
import numpy as np
import torch

import oracle
import parity
from oracle import free as F
from paper_2609_21803_amd import instances as I
from paper_2609_21803_amd import native

timed = sys.argv[1:] == ["timed"]
ROUND32 = 1 | 2 | 4 | 8
f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
orders = [F.key_modes(int(k)) for k in F.seed(6)]
x0, goal, inst = I.push_free_pairs(5400, 8)
pair = np.repeat(np.arange(8), len(orders))
split = lambda K: [50 // K + (1 if j < 50 % K else 0) for j in range(K)]
knots = [split(len(o)) if timed else [10] * len(o) for o in orders] * 8
b = I.orders_batch(x0, goal, inst, pair, orders * 8, knots)
ctx = native.Context(max_batch=len(b["nseg"]), max_segments=6, max_intervals=60,
                     task=native.TASK_PUSH_FREE_TIMED if timed else native.TASK_PUSH_FREE)
print("step: gpu launch", flush=True)
out = ctx.evaluate(**native.to_device(b), want_traj=False)
torch.cuda.synchronize()
ctx.check()
g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
print("step: oracle on all orders", flush=True)
t0 = time.time()
parts = []
n = len(b["nseg"])
for c0 in range(0, n, 7380):
    sl = slice(c0, min(n, c0 + 7380))
    parts.append(F.evaluate(f32(b["x0"][sl]), f32(b["goal"][sl]), f32(b["inst"][sl]), b["nseg"][sl], b["modes"][sl],
                            b["knots"][sl], nmax=60, timed=timed))
    print(f"  oracle {sl.stop}/{n} after {time.time() - t0:.0f} s", flush=True)
o = {k: np.concatenate([p[k] for p in parts]) for k in ("cost", "viol", "feasible", "stats")}
print(f"oracle {time.time() - t0:.1f} s", flush=True)


def solve(sub, rows, r32):
    return F.evaluate(f32(sub["x0"]), f32(sub["goal"]), f32(sub["inst"]), sub["nseg"], sub["modes"], sub["knots"],
                      params=oracle.Params(round32=r32), nmax=60, timed=timed)


parity.check(g, o, b, solve, "free" + (" timed" if timed else "") + ", all 118,080", round32=ROUND32,
             allow=2e-3 if timed else 1e-3)
print("done", flush=True)

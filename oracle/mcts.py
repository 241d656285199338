"""Oracle of the MCTS allocation policy of the ablations (UCT with c = 0.8, virtual loss,
random rollouts; pool of P orders per update), over the evaluator oracles.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading of the policy (the paper names its parts but not their details):
* the tree is over order prefixes; a node of length d has the actions "stop" (d >= 1: the
  prefix itself is the order) and "append id" (d < kcap) for every id, in id order, that
  keeps the prefix in the task's language;
* one batch selects P orders: from the root, a node with untried actions expands the first
  one (stop before ids) and the walk ends at the new child; otherwise it moves to the child
  of largest W/N + c sqrt(ln N_parent / N) (first in action order on ties); every node on
  the path gets a virtual visit (N += 1) at once, so later selections of the batch spread;
* the rollout from a new "append" child of length d draws K = d + out(8r) mod (kcap - d + 1)
  and appends, for j = d .. K-1, admissible id number out(8r+1+j) mod (count) in id order
  (stopping early when no id is admissible); r counts rollouts from 0; out() is the
  SplitMix64 stream of `sample.py`;
* evaluated orders are cached: a repeated order takes its stored result, and the budget
  counts distinct evaluated orders (a batch stops selecting when its new orders would
  exceed the remaining budget); the search ends at the budget, when a batch brings no new
  order and no node has an untried action left (the whole language is evaluated), or after
  STALL consecutive batches without a new order;
* after the batch is evaluated the best value so far is updated, then every selection's
  path adds the reward (W += r): pushing, J_best / J for a feasible order and 0 otherwise;
  flipping, M_best / M with the merit M = J + mu max(v - eps, 0) (0 if not finite);
* refinement and the returned plan are the expansion's (the k_ref best feasible by (J, key)).
"""
from __future__ import annotations

import math

import numpy as np

from .sample import _evaluate, key_make, key_modes, splitmix64

STALL = 64


class Node:
    __slots__ = ("prefix", "stop", "untried", "children", "N", "W")

    def __init__(self, prefix, stop, actions):
        self.prefix = prefix
        self.stop = stop
        self.untried = actions
        self.children = []          # (action, node) in action order
        self.N = 0
        self.W = 0.0


class Tree:
    def __init__(self, task, kcap, c=0.8, seed=0):
        self.task, self.kcap, self.c, self.seed = task, kcap, c, seed
        if task == 1:
            from . import flip as F
            self.adm, self.M = F.admissible, 845
        else:
            self.adm, self.M = (lambda m: True), 12
        self.untried = 0                # untried actions over the whole tree
        self.root = self.node((), False)
        self.rollouts = 0

    def node(self, prefix, stop):
        n = Node(prefix, stop, [] if stop else self.actions(prefix))
        self.untried += len(n.untried)
        return n

    def ids_after(self, prefix):
        return [a for a in range(self.M) if self.adm(list(prefix) + [a])]

    def actions(self, prefix):
        acts = [-1] if len(prefix) >= 1 else []              # -1 = stop
        if len(prefix) < self.kcap:
            acts += self.ids_after(prefix)
        return acts

    def uct(self, parent, child):
        return child.W / child.N + self.c * math.sqrt(math.log(parent.N) / child.N)

    def select(self):
        node, path = self.root, [self.root]
        while True:
            if node.untried:
                a = node.untried.pop(0)
                self.untried -= 1
                child = self.node(node.prefix, True) if a == -1 else self.node(node.prefix + (a,), False)
                node.children.append((a, child))
                path.append(child)
                break
            if not node.children:
                break
            best, bval = None, -math.inf
            for _, ch in node.children:
                v = self.uct(node, ch)
                if v > bval:
                    best, bval = ch, v
            node = best
            path.append(node)
        leaf = path[-1]
        order = list(leaf.prefix) if leaf.stop else self.rollout(list(leaf.prefix))
        for n in path:
            n.N += 1
        return path, order

    def rollout(self, prefix):
        r = self.rollouts
        self.rollouts += 1
        d = len(prefix)
        if d >= self.kcap:
            return prefix
        K = d + splitmix64(self.seed, 8 * r) % (self.kcap - d + 1)
        m = list(prefix)
        for j in range(d, K):
            cand = self.ids_after(m)
            if not cand:
                break
            m.append(cand[splitmix64(self.seed, 8 * r + 1 + j) % len(cand)])
        return m


def mcts_search(task, x0, goal, inst, kcap, P, eval_budget, seed, knots_per_segment, k_ref, c=0.8, mu_merit=100.0,
                params=None, ref_params=None, max_batches=10 ** 6, evaluate=None):
    """Returns (best key or 0, refined J, refined v, evaluated keys in evaluation order,
    their J, v, number of batches, the tree).  `evaluate(keys, refine) -> (J, v)` replaces the
    evaluator oracle (for the pins of the search logic)."""
    import oracle
    params = params or oracle.Params()
    ref_params = ref_params or oracle.Params(**{**params.__dict__, **oracle.REFINE})
    if evaluate is None:
        evaluate = lambda ks, refine: _evaluate(task, ks, x0, goal, inst, knots_per_segment,
                                                ref_params if refine else params)
    eps = params.eps_feas
    tree = Tree(task, kcap, c, seed)
    cache = {}
    keys, Js, vs = [], [], []
    best = math.inf                 # J_best (pushing) or M_best (flipping)
    batches = stall = 0
    while len(keys) < eval_budget and batches < max_batches:
        sel, new = [], []
        for _ in range(P):
            path, order = tree.select()
            k = key_make(order)
            if k not in cache and k not in new:
                if len(keys) + len(new) >= eval_budget:
                    for n in path:                      # undo: this selection is not taken
                        n.N -= 1
                    break
                new.append(k)
            sel.append((path, k))
        batches += 1
        if new:
            J, v = evaluate(new, False)
            for k, a, b in zip(new, J, v):
                cache[k] = (a, b)
                keys.append(k)
                Js.append(a)
                vs.append(b)
                if task == 1:
                    M = a + mu_merit * max(b - eps, 0.0) if (np.isfinite(a) and np.isfinite(b)) else math.inf
                    best = min(best, M)
                elif b <= eps and np.isfinite(a):
                    best = min(best, a)
        for path, k in sel:
            a, b = cache[k]
            if task == 1:
                M = a + mu_merit * max(b - eps, 0.0) if (np.isfinite(a) and np.isfinite(b)) else math.inf
                rew = best / M if (math.isfinite(M) and M > 0) else 0.0
            else:
                rew = best / a if (b <= eps and np.isfinite(a) and a > 0) else 0.0
            for n in path:
                n.W += rew
        stall = 0 if new else stall + 1
        if not new and (tree.untried == 0 or stall >= STALL):
            break
    feas = sorted((Js[i], keys[i]) for i in range(len(keys)) if vs[i] <= eps and np.isfinite(Js[i]))
    ref = [k for _, k in feas[:k_ref]]
    out = (0, np.nan, np.inf)
    if ref:
        J, v = evaluate(ref, True)
        for k, a, b in zip(ref, J, v):
            if b <= ref_params.eps_feas and np.isfinite(a):
                if out[0] == 0 or a < out[1] or (a == out[1] and k < out[0]):
                    out = (k, a, b)
    return out[0], out[1], out[2], keys, np.array(Js), np.array(vs), batches, tree


def first_batch(task, kcap, P, seed, eval_budget=10 ** 9):
    """The distinct orders of the first batch in selection order (no evaluation needed)."""
    tree = Tree(task, kcap, 0.8, seed)
    new = []
    for _ in range(P):
        path, order = tree.select()
        k = key_make(order)
        if k not in new:
            if len(new) >= eval_budget:
                break
            new.append(k)
    return new

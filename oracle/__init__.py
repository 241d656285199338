"""FP64 CPU oracle of the mode-conditioned TO evaluator and the greedy mode expansion.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code with
the HIP library in ``paper_2609_21803_amd`` and never imports it.

The numerical work lives in ``comet_oracle.c`` (plain C, FP64, ``-ffp-contract=off``);
this module only marshals NumPy arrays through ctypes.  Beside it: ``flip.py`` /
``flip_oracle.c`` (bimanual flipping), ``free.py`` / ``free_oracle.c`` (pushing with free
motion, built with and without optimised timing), ``sample.py`` and ``mcts.py`` (the
ablations' allocation policies) and ``mlp.py`` (the NumPy oracle of the learned proposal
network).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "comet_oracle.c")
_LIB = os.path.join(_HERE, "libcomet_oracle.so")

MAXSEG = 6
N_TYPES = 13


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11", "-fPIC", "-shared",
             "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class SolverParams(C.Structure):
    _fields_ = [("al_max", C.c_int32), ("gn_max", C.c_int32), ("chol_retries", C.c_int32),
                ("ls_trials", C.c_int32), ("max_rejects", C.c_int32), ("timed", C.c_int32), ("mu0", C.c_double), ("mu_min", C.c_double),
                ("rho0", C.c_double), ("rho_min", C.c_double), ("rho_max", C.c_double),
                ("armijo_c1", C.c_double), ("eta_star", C.c_double), ("omega_star", C.c_double),
                ("rc_star", C.c_double), ("eps_feas", C.c_double),
                ("mu0_warm", C.c_double), ("round32", C.c_int32)]


class ExpandParams(C.Structure):
    _fields_ = [("kcap", C.c_int32), ("seed_max_segments", C.c_int32), ("radius", C.c_int32),
                ("rounds", C.c_int32), ("frontier_W", C.c_int32), ("knots_per_segment", C.c_int32),
                ("k_ref", C.c_int32), ("n_total", C.c_int32), ("batch_B", C.c_int64),
                ("eval_budget", C.c_int64), ("mu_merit", C.c_double)]


@dataclass
class Params:
    """Solver parameters (same names and defaults as the library's)."""
    al_max: int = 20
    gn_max: int = 10
    chol_retries: int = 6
    ls_trials: int = 8
    max_rejects: int = 4
    timed: int = 0          # 1: the optimised-timing pushing problem (durations are controls)
    mu0: float = 1e-2
    mu_min: float = 1e-4
    rho0: float = 1e-4
    rho_min: float = 1e-8
    rho_max: float = 1e8
    armijo_c1: float = 1e-4
    eta_star: float = 1e-6
    omega_star: float = 1e-4
    rc_star: float = 1e-6
    eps_feas: float = 1e-5
    mu0_warm: float = 1e-4
    # test switch (0 = plain FP64): round to float32 the step direction (1), the multipliers
    # (2), the scaled row Jacobians (4), the gains with the forward recursion in float32 (8),
    # the gains alone (16); results with bits set are perturbations, not the oracle's answer
    round32: int = 0

    def c(self) -> SolverParams:
        return SolverParams(*[getattr(self, f) for f, _ in SolverParams._fields_])


REFINE = dict(al_max=40, gn_max=25)

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.oracle_evaluate.argtypes = [C.c_int64, C.c_int32, C.c_int32, P, P, P, P, P, P, P,
                                      C.POINTER(SolverParams), C.c_int32, P, P, P, P, P]
        L.oracle_evaluate.restype = C.c_int
        I = C.c_int32
        L.oracle_push_scales.argtypes = [I, P]
        L.oracle_push_rows.argtypes = [I, I, I, I, C.c_double, P, P, P, P]
        L.oracle_push_cost.argtypes = [I, P, P, P]
        L.oracle_push_cost.restype = C.c_double
        L.oracle_push_initial.argtypes = [I, I, P, P, P, P, C.c_double, P]
        L.oracle_push_merit.argtypes = [I, I, P, P, P, P, C.c_double, P, P, P, P, C.c_double, P, P]
        L.oracle_push_step.argtypes = [I, I, P, P, P, P, C.c_double, P, P, P, P, C.c_double, C.c_double, P]
        L.oracle_push_blocks.argtypes = [I, I, P, P, P, P, C.c_double, P, P, P, P, P, P]
        L.oracle_push_score.argtypes = [I, I, P, P, P, P, C.c_double, P, P, P]
        L.oracle_neighbours.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, P]
        L.oracle_neighbours.restype = C.c_int64
        L.oracle_expand.argtypes = [P, P, C.c_double, C.POINTER(ExpandParams), C.POINTER(SolverParams),
                                    C.POINTER(SolverParams), C.c_int32, P, P, P, P, P, P, P, C.c_int64]
        L.oracle_expand_next.argtypes = [C.c_int64, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int64, P]
        L.oracle_expand_next.restype = C.c_int64
        L.oracle_merit.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.oracle_merit.restype = C.c_double
        L.oracle_enumerate.argtypes = [P, P, C.c_double, C.c_int32, C.POINTER(ExpandParams),
                                       C.POINTER(SolverParams), C.POINTER(SolverParams), C.c_int32, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def default_threads() -> int:
    return int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))


def evaluate(x0, goal, inst, nseg, modes, knots, params: Params | None = None, warm=None,
             nmax: int | None = None, nthreads: int | None = None):
    """Solve one TO per sequence.  Returns dict(cost, viol, feasible, traj, stats)."""
    params = params or Params()
    x0, goal, inst = _f64(x0), _f64(goal), _f64(inst).reshape(-1)
    nseg, modes, knots = _i32(nseg), _i32(modes), _i32(knots)
    B, smax = modes.shape
    if smax != MAXSEG:
        m2 = np.zeros((B, MAXSEG), np.int32)
        k2 = np.zeros((B, MAXSEG), np.int32)
        m2[:, :smax] = modes
        k2[:, :smax] = knots
        modes, knots, smax = m2, k2, MAXSEG
    if nmax is None:
        nmax = int(max(1, (knots * (np.arange(MAXSEG)[None, :] < nseg[:, None])).sum(1).max(initial=1)))
    cost = np.zeros(B)
    viol = np.zeros(B)
    feas = np.zeros(B, np.uint8)
    traj = np.zeros((B, nmax + 1, 8 if params.timed else 7))
    stats = np.zeros((B, 4), np.int32)
    w = None if warm is None else _f64(warm)
    prm = params.c()
    rc = lib().oracle_evaluate(B, smax, nmax, _p(x0), _p(goal), _p(inst), _p(nseg), _p(modes), _p(knots),
                               _p(w), C.byref(prm), nthreads or default_threads(), _p(cost), _p(viol),
                               _p(feas), _p(traj), _p(stats))
    if rc != 0:
        raise ValueError("oracle_evaluate rejected its arguments")
    return dict(cost=cost, viol=viol, feasible=feas, traj=traj, stats=stats)


def scales(timed: int = 0) -> np.ndarray:
    """Row scales of the fixed-step (timed=0) or optimised-timing (timed=1) pushing
    problem; the last type (duration bounds) exists only with optimised timing."""
    out = np.zeros(N_TYPES)
    lib().oracle_push_scales(int(timed), _p(out))
    return out


def push_rows(face, slip, smask, mu, v, timed: int = 0):
    """Rows of one interval: v = (x_k, u_k, x_{k+1}) with 11 entries (12 with timing)."""
    nr, nv = (12, 12) if timed else (10, 11)
    v = _f64(v)
    c = np.zeros(nr)
    J = np.zeros((nr, nv))
    en = np.zeros(nr, np.int32)
    lib().oracle_push_rows(int(timed), face, slip, smask, mu, _p(v), _p(c), _p(J), _p(en))
    return c, J, en


def push_cost(u, timed: int = 0):
    """Stage cost, its gradient and its Hessian model (full nu x nu)."""
    nu = 4 if timed else 3
    u = _f64(u)
    g = np.zeros(nu)
    H = np.zeros((nu, nu))
    J = lib().oracle_push_cost(int(timed), _p(u), _p(g), _p(H))
    return J, g, H


class Seq:
    """One mode-conditioned problem for the single-sequence debug entry points."""

    def __init__(self, modes, knots, x0=(0, 0, 0, 0), goal=(0, 0, 0), mu=0.4, timed=0):
        self.timed = int(timed)
        self.nw, self.nr, self.nv, self.ni = (8, 12, 12, 7) if self.timed else (7, 10, 11, 5)
        self.modes = _i32(modes)
        self.knots = _i32(knots)
        self.nseg = len(self.modes)
        self.x0 = _f64(x0)
        self.goal = _f64(goal)
        self.mu = float(mu)
        self.N = int(self.knots.sum())

    def _a(self):
        return (self.timed, self.nseg, _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal), self.mu)

    def initial(self):
        z = np.zeros(self.N * self.nw)
        lib().oracle_push_initial(*self._a(), _p(z))
        return z

    def duals(self):
        return np.zeros(self.N * 5), np.zeros(self.N * self.ni), np.zeros(3)

    def merit(self, z, lam, nu, lamT, mu_al):
        phi = C.c_double()
        g = np.zeros(self.N * self.nw)
        z, lam, nu, lamT = _f64(z), _f64(lam), _f64(nu), _f64(lamT)
        lib().oracle_push_merit(*self._a(), _p(z), _p(lam), _p(nu), _p(lamT), mu_al, C.byref(phi), _p(g))
        return phi.value, g

    def step(self, z, lam, nu, lamT, mu_al, rho):
        dz = np.zeros(self.N * self.nw)
        z, lam, nu, lamT = _f64(z), _f64(lam), _f64(nu), _f64(lamT)
        ok = lib().oracle_push_step(*self._a(), _p(z), _p(lam), _p(nu), _p(lamT), mu_al, rho, _p(dz))
        return (dz if ok > 0 else None)

    def blocks(self, z):
        N = self.N
        c = np.zeros((N, self.nr))
        J = np.zeros((N, self.nr, self.nv))
        en = np.zeros((N, self.nr), np.int32)
        cT = np.zeros(3)
        JT = np.zeros((3, 4))
        z = _f64(z)
        lib().oracle_push_blocks(*self._a(), _p(z), _p(c), _p(J), _p(en), _p(cT), _p(JT))
        return c, J, en, cT, JT

    def score(self, z):
        J = C.c_double()
        v = C.c_double()
        z = _f64(z)
        lib().oracle_push_score(*self._a(), _p(z), C.byref(J), C.byref(v))
        return J.value, v.value


def key_make(modes) -> int:
    k = len(modes) << 60
    for i, m in enumerate(modes):
        k |= int(m) << (50 - 10 * i)
    return k


def key_modes(key: int):
    K = key >> 60
    return [(key >> (50 - 10 * i)) & 1023 for i in range(K)]


def neighbours(modes, n_modes=12, kcap=6, radius=1):
    out = np.zeros(1_000_000, np.uint64)
    n = lib().oracle_neighbours(key_make(modes), n_modes, kcap, radius, _p(out))
    return [int(k) for k in out[:n]]


@dataclass
class Expand:
    kcap: int = 3
    seed_max_segments: int = 2
    radius: int = 1
    rounds: int = 8
    frontier_W: int = 4096
    knots_per_segment: int = 8
    k_ref: int = 64
    n_total: int = 24
    batch_B: int = 131072
    eval_budget: int = 200000
    mu_merit: float = 100.0

    def c(self) -> ExpandParams:
        return ExpandParams(*[getattr(self, f) for f, _ in ExpandParams._fields_])


def expand(x0, goal, mu, ep: Expand, params: Params | None = None, refine: Params | None = None,
           nthreads=None, eval_cap=0):
    params = params or Params()
    refine = refine or Params(**{**params.__dict__, **REFINE})
    x0, goal = _f64(x0), _f64(goal)
    key = C.c_uint64()
    J = C.c_double()
    v = C.c_double()
    ctr = np.zeros(4, np.int64)
    ek = np.zeros(max(eval_cap, 1), np.uint64)
    eJ = np.zeros(max(eval_cap, 1))
    ev = np.zeros(max(eval_cap, 1))
    epc, p1, p2 = ep.c(), params.c(), refine.c()
    lib().oracle_expand(_p(x0), _p(goal), float(mu), C.byref(epc), C.byref(p1), C.byref(p2),
                        nthreads or default_threads(), C.byref(key), C.byref(J), C.byref(v), _p(ctr),
                        _p(ek), _p(eJ), _p(ev), eval_cap)
    n = int(min(ctr[0], eval_cap))
    return dict(best_key=int(key.value), best_cost=J.value, best_viol=v.value, evaluated=int(ctr[0]),
                rounds=int(ctr[1]), n_feasible=int(ctr[2]), first_feasible=int(ctr[3]),
                eval_keys=[int(k) for k in ek[:n]], eval_cost=eJ[:n].copy(), eval_viol=ev[:n].copy())


def enumerate_all(x0, goal, mu, ep: Expand, kmin=1, params: Params | None = None, refine: Params | None = None,
                  nthreads=None):
    params = params or Params()
    refine = refine or Params(**{**params.__dict__, **REFINE})
    x0, goal = _f64(x0), _f64(goal)
    key = C.c_uint64()
    J = C.c_double()
    v = C.c_double()
    n = C.c_int64()
    epc, p1, p2 = ep.c(), params.c(), refine.c()
    lib().oracle_enumerate(_p(x0), _p(goal), float(mu), kmin, C.byref(epc), C.byref(p1), C.byref(p2),
                           nthreads or default_threads(), C.byref(key), C.byref(J), C.byref(v), C.byref(n))
    return dict(best_key=int(key.value), best_cost=J.value, best_viol=v.value, evaluated=int(n.value))


def merit(J: float, v: float, eps: float = 1e-5, mu_merit: float = 100.0) -> float:
    """Eq. (5) merit of one evaluated order (NaN -> +inf), as the expansion ranks it."""
    return float(lib().oracle_merit(float(J), float(v), float(eps), float(mu_merit)))


def expand_next(keys, merit, n_modes=12, kcap=3, radius=1, frontier_W=4096, room=131072):
    """One batch-construction step of Alg. 1 on given (key, merit) pairs."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    merit = _f64(merit)
    out = np.zeros(max(int(room), 1), np.uint64)
    n = lib().oracle_expand_next(len(keys), _p(keys), _p(merit), n_modes, kcap, radius, frontier_W, int(room), _p(out))
    return out[:n].copy()

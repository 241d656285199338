"""FP64 CPU oracle of the bimanual flipping TO and its mode language (ctypes wrapper).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The numerical work lives in
``flip_oracle.c``; this module marshals NumPy arrays.

Layouts: x0 [B, 8] = (px, py, th, vx, vy, om, s1, s2); goal [B, 2] = (px, th); inst [B]
= table friction; modes / knots [B, 6]; trajectory rows (x_k, u_k) of 17 values with
u = (ax, ay, al, f1n, f1t, sd1, f2n, f2t, sd2).  Mode id = (f1 * 13 + f2) * 5 + g.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import Params, default_threads

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flip_oracle.c")
_LIB = os.path.join(_HERE, "libflip_oracle.so")

NX, NU, NW, NV, NE, NI, NR, NT = 8, 9, 17, 25, 17, 15, 32, 5
MAXSEG = 6
N_MODES = 845
X0 = np.array([0.0, 0.05, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])   # at rest on the long face


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11", "-fPIC", "-shared",
             "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        from . import ExpandParams, SolverParams
        L = C.CDLL(build())
        P = C.c_void_p
        L.flip_evaluate.argtypes = [C.c_int64, C.c_int32, C.c_int32, P, P, P, P, P, P, P,
                                    C.POINTER(SolverParams), C.c_int32, P, P, P, P, P]
        L.flip_rows_at.argtypes = [C.c_int32, P, P, P, P, C.c_double, C.c_int32, P, P, P, P]
        L.flip_rows_real.argtypes = [C.c_int32, P, P, P, P, C.c_double, C.c_int32, P, P, P]
        L.flip_setup_info.argtypes = [C.c_int32, P, P, P, P, P]
        L.flip_initial.argtypes = [C.c_int32, P, P, P, P, C.c_double, P]
        L.flip_merit_grad_step.argtypes = [C.c_int32, P, P, P, P, C.c_double, P, P, P, P, C.c_double, C.c_double,
                                           P, P, P]
        L.flip_score.argtypes = [C.c_int32, P, P, P, P, C.c_double, P, P, P]
        L.flip_admissible.argtypes = [C.c_int32, P]
        L.flip_seed.argtypes = [C.c_int32, C.c_int64, P]
        L.flip_seed.restype = C.c_int64
        L.flip_expand_next.argtypes = [C.c_int64, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int64, P]
        L.flip_expand_next.restype = C.c_int64
        L.flip_expand.argtypes = [P, P, C.c_double, C.POINTER(ExpandParams), C.POINTER(SolverParams),
                                  C.POINTER(SolverParams), C.c_int32, P, P, P, P, P, P, P, C.c_int64]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def mode_id(f1: int, f2: int, g: int) -> int:
    return (f1 * 13 + f2) * 5 + g


def finger(face: int, slip: int) -> int:
    """finger code of a contact on `face` with slip 0 stick, 1 slide+, 2 slide-"""
    return 1 + 3 * face + slip


def evaluate(x0, goal, inst, nseg, modes, knots, params: Params | None = None, warm=None, nmax=None,
             nthreads=None):
    params = params or Params()
    x0, goal, inst = _f64(x0), _f64(goal), _f64(inst).reshape(-1)
    nseg, modes, knots = _i32(nseg), _i32(modes), _i32(knots)
    B, smax = modes.shape
    if smax != MAXSEG:
        m2 = np.zeros((B, MAXSEG), np.int32)
        k2 = np.zeros((B, MAXSEG), np.int32)
        m2[:, :smax], k2[:, :smax] = modes, knots
        modes, knots, smax = m2, k2, MAXSEG
    if nmax is None:
        nmax = int(max(1, (knots * (np.arange(MAXSEG)[None, :] < nseg[:, None])).sum(1).max(initial=1)))
    cost, viol = np.zeros(B), np.zeros(B)
    feas = np.zeros(B, np.uint8)
    traj = np.zeros((B, nmax + 1, NX + NU))
    stats = np.zeros((B, 4), np.int32)
    w = None if warm is None else _f64(warm)
    prm = params.c()
    rc = lib().flip_evaluate(B, smax, nmax, _p(x0), _p(goal), _p(inst), _p(nseg), _p(modes), _p(knots), _p(w),
                             C.byref(prm), nthreads or default_threads(), _p(cost), _p(viol), _p(feas), _p(traj),
                             _p(stats))
    if rc != 0:
        raise ValueError("flip_evaluate rejected its arguments")
    return dict(cost=cost, viol=viol, feasible=feas, traj=traj, stats=stats)


class Seq:
    """One flip order on one instance, for the pins."""

    def __init__(self, modes, knots, goal=(0.0, np.pi / 2), mu_g=0.7, x0=X0):
        self.K = len(modes)
        self.modes = _i32(list(modes) + [0] * (MAXSEG - len(modes)))
        self.knots = _i32(list(knots) + [0] * (MAXSEG - len(knots)))
        self.x0, self.goal, self.mu_g = _f64(x0), _f64(goal), float(mu_g)
        self.N = int(sum(knots))

    def rows(self, k, v, complex_step=True):
        c = np.zeros(NR)
        en = np.zeros(NR, np.int32)
        v = _f64(v)
        if complex_step:
            J = np.zeros((NR, NV))
            rc = lib().flip_rows_at(self.K, _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal), self.mu_g,
                                    k, _p(v), _p(c), _p(J), _p(en))
            assert rc == 0
            return c, J, en
        rc = lib().flip_rows_real(self.K, _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal), self.mu_g, k,
                                  _p(v), _p(c), _p(en))
        assert rc == 0
        return c, en

    def info(self):
        info = np.zeros((self.N, 6), np.int32)
        ths = np.zeros(self.N)
        n = C.c_int32()
        assert lib().flip_setup_info(self.K, _p(self.modes), _p(self.knots), _p(info), _p(ths), C.byref(n)) == 0
        return info, ths

    def initial(self):
        z = np.zeros(self.N * NW)
        assert lib().flip_initial(self.K, _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal), self.mu_g,
                                  _p(z)) == 0
        return z

    def merit_grad_step(self, z, lam, nu, lamT, mu, rho):
        phi = C.c_double()
        g = np.zeros(self.N * NW)
        dz = np.zeros(self.N * NW)
        rc = lib().flip_merit_grad_step(self.K, _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal),
                                        self.mu_g, _p(_f64(z)), _p(_f64(lam)), _p(_f64(nu)), _p(_f64(lamT)), mu, rho,
                                        C.byref(phi), _p(g), _p(dz))
        return phi.value, g, (dz if rc == 0 else None)

    def score(self, z):
        J, v = C.c_double(), C.c_double()
        assert lib().flip_score(self.K, _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal), self.mu_g,
                                _p(_f64(z)), C.byref(J), C.byref(v)) == 0
        return J.value, v.value

    def args(self, z, k):
        """(x_k, u_k, x_{k+1}) of interval k from the primal z"""
        xk = self.x0 if k == 0 else z[(k - 1) * NW + NU:(k - 1) * NW + NW]
        return np.concatenate([xk, z[k * NW:(k + 1) * NW]])


def admissible(modes) -> bool:
    m = _i32(list(modes))
    return bool(lib().flip_admissible(len(m), _p(m)))


def key_make(modes) -> int:
    k = len(modes) << 60
    for i, m in enumerate(modes):
        k |= int(m) << (50 - 10 * i)
    return k


def key_modes(k: int):
    return [(k >> (50 - 10 * i)) & 1023 for i in range(k >> 60)]


def seed(kmax: int, cap: int = 10 ** 7) -> np.ndarray:
    out = np.zeros(min(cap, 10 ** 7), np.uint64)
    n = lib().flip_seed(kmax, len(out), _p(out))
    return out[:n]


def expand_next(keys, merit, kcap, radius, W, room) -> np.ndarray:
    keys = np.ascontiguousarray(keys, np.uint64)
    merit = _f64(merit)
    out = np.zeros(max(room, 1), np.uint64)
    n = lib().flip_expand_next(len(keys), _p(keys), _p(merit), kcap, radius, W, room, _p(out))
    return out[:n]


def expand(x0, goal, mu_g, ep, params=None, ref_params=None, nthreads=None, eval_cap=200000):
    """Greedy expansion with refinement on one instance; returns (best_key, J, v,
    counters, evaluated keys, their J, v)."""
    from . import REFINE, Params
    params = params or Params()
    ref_params = ref_params or Params(**{**params.__dict__, **REFINE})
    bk = C.c_uint64()
    bJ, bv = C.c_double(), C.c_double()
    cnt = np.zeros(4, np.int64)
    ek = np.zeros(eval_cap, np.uint64)
    eJ, ev = np.zeros(eval_cap), np.zeros(eval_cap)
    pe, pr, epc = params.c(), ref_params.c(), ep.c()
    lib().flip_expand(_p(_f64(x0)), _p(_f64(goal)), float(mu_g), C.byref(epc), C.byref(pe), C.byref(pr),
                      nthreads or default_threads(), C.byref(bk), C.byref(bJ), C.byref(bv), _p(cnt), _p(ek), _p(eJ),
                      _p(ev), eval_cap)
    n = int(min(cnt[0], eval_cap))
    return bk.value, bJ.value, bv.value, cnt, ek[:n], eJ[:n], ev[:n]

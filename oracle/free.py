"""FP64 CPU oracle of planar pushing with free-motion segments and its mode language
(ctypes wrapper).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The numerical work lives in
``free_oracle.c``; this module marshals NumPy arrays.

Layouts: x0 [B, 5] = (x, y, theta, p_x, p_y), the pusher in the slider frame; goal [B, 3]
= (x, y, theta); inst [B] = pusher friction; modes / knots [B, smax <= 8]; trajectory rows
(x_k, u_k) of 9 values with u = (F_n, F_t, v_x, v_y), the pusher velocity in the slider
frame.  Mode ids 0..11: contact on face id // 3 with slip id % 3 (stick, slide+, slide-);
12..15: free motion in front of face id - 12.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import Params, default_threads

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "free_oracle.c")
_LIB = os.path.join(_HERE, "libfree_oracle.so")

NX, NU, NW, NV, NE, NI, NR, NT = 5, 4, 9, 14, 8, 7, 15, 3
MAXSEG = 8
N_MODES = 16
N_TYPES = 16
# slider at rest at the origin, pusher 3 cm in front of face 3 (below the slider)
X0 = np.array([0.0, 0.0, 0.0, 0.0, -0.08])


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
        from . import SolverParams
        L = C.CDLL(build())
        P = C.c_void_p
        L.free_evaluate.argtypes = [C.c_int64, C.c_int32, C.c_int32, P, P, P, P, P, P, P,
                                    C.POINTER(SolverParams), C.c_int32, P, P, P, P, P]
        L.free_scales.argtypes = [P]
        L.free_rows.argtypes = [C.c_int32, C.c_double, P, P, P, P, P]
        L.free_cost.argtypes = [P, P]
        L.free_cost.restype = C.c_double
        L.free_initial.argtypes = [C.c_int32, P, P, P, P, C.c_double, P]
        L.free_score.argtypes = [C.c_int32, P, P, P, P, C.c_double, P, P, P]
        L.free_merit_grad_step.argtypes = [C.c_int32, P, P, P, P, C.c_double, P, P, P, P, C.c_double, C.c_double,
                                           P, P, P]
        L.free_admissible.argtypes = [C.c_int32, P]
        L.free_neighbours.argtypes = [C.c_uint64, C.c_int32, C.c_int32, P]
        L.free_neighbours.restype = C.c_int64
        L.free_seed.argtypes = [C.c_int32, C.c_int64, P]
        L.free_seed.restype = C.c_int64
        L.free_expand_next.argtypes = [C.c_int64, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int64, P]
        L.free_expand_next.restype = C.c_int64
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def contact(face: int, slip: int) -> int:
    return 3 * face + slip


def free(region: int) -> int:
    return 12 + region


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
    rc = lib().free_evaluate(B, smax, nmax, _p(x0), _p(goal), _p(inst), _p(nseg), _p(modes), _p(knots), _p(w),
                             C.byref(prm), nthreads or default_threads(), _p(cost), _p(viol), _p(feas), _p(traj),
                             _p(stats))
    if rc != 0:
        raise ValueError("free_evaluate rejected its arguments")
    return dict(cost=cost, viol=viol, feasible=feas, traj=traj, stats=stats)


def scales() -> np.ndarray:
    out = np.zeros(N_TYPES)
    lib().free_scales(_p(out))
    return out


def rows(mode: int, mu: float, v):
    """Rows of one interval at v = (x_k, u_k, x_{k+1}) in physical units: (c, J, en, type)."""
    v = _f64(v)
    c, J = np.zeros(NR), np.zeros((NR, NV))
    en, ty = np.zeros(NR, np.int32), np.zeros(NR, np.int32)
    if lib().free_rows(int(mode), float(mu), _p(v), _p(c), _p(J), _p(en), _p(ty)) != 0:
        raise ValueError("bad mode")
    return c, J, en, ty


def cost(u):
    u = _f64(u)
    g = np.zeros(NU)
    return lib().free_cost(_p(u), _p(g)), g


class Seq:
    """One order on one instance, for the pins."""

    def __init__(self, modes, knots, goal=(0.1, 0.1, np.pi / 4), mu=0.4, x0=X0):
        self.modes, self.knots = _i32(modes), _i32(knots)
        self.goal, self.mu, self.x0 = _f64(goal), float(mu), _f64(x0)
        self.N = int(self.knots.sum())

    def initial(self):
        z = np.zeros(self.N * NW)
        n = lib().free_initial(len(self.modes), _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal), self.mu,
                               _p(z))
        if n < 0:
            raise ValueError("bad order")
        return z

    def score(self, z):
        J, v = C.c_double(), C.c_double()
        if lib().free_score(len(self.modes), _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal), self.mu,
                            _p(_f64(z)), C.byref(J), C.byref(v)) != 0:
            raise ValueError("bad order")
        return J.value, v.value

    def merit_grad_step(self, z, lam, nu, lamT, mu, rho):
        phi = C.c_double()
        g, dz = np.zeros(self.N * NW), np.zeros(self.N * NW)
        rc = lib().free_merit_grad_step(len(self.modes), _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal),
                                        self.mu, _p(_f64(z)), _p(_f64(lam)), _p(_f64(nu)), _p(_f64(lamT)), float(mu),
                                        float(rho), C.byref(phi), _p(g), _p(dz))
        return phi.value, g, dz, rc == 0

    def args(self, z, k):
        """v = (x_k, u_k, x_{k+1}) of interval k"""
        z = _f64(z).reshape(self.N, NW)
        xk = self.x0 if k == 0 else z[k - 1, NU:]
        return np.concatenate([xk, z[k, :NU], z[k, NU:]])

    def mode_of(self, k):
        return int(np.repeat(self.modes, self.knots)[k])


def admissible(modes) -> bool:
    m = _i32(list(modes))
    return bool(lib().free_admissible(len(m), _p(m)))


def key_make(modes) -> int:
    """K << 60 | m_0 << 56 | m_1 << 52 | ... (4 bits per id, up to 8 segments)"""
    k = len(modes) << 60
    for i, m in enumerate(modes):
        k |= int(m) << (56 - 4 * i)
    return k


def key_modes(k: int):
    return [(int(k) >> (56 - 4 * i)) & 15 for i in range(int(k) >> 60)]


def neighbours(key: int, kcap: int, radius: int) -> np.ndarray:
    out = np.zeros(260 * 260 + 16, np.uint64)
    n = lib().free_neighbours(int(key), kcap, radius, _p(out))
    return out[:n]


def seed(kmax: int, cap: int = 10 ** 7) -> np.ndarray:
    out = np.zeros(min(cap, 10 ** 7), np.uint64)
    n = lib().free_seed(kmax, len(out), _p(out))
    return out[:n]


def expand_next(keys, merit, kcap, radius, W, room) -> np.ndarray:
    keys = np.ascontiguousarray(keys, np.uint64)
    merit = _f64(merit)
    out = np.zeros(max(room, 1), np.uint64)
    n = lib().free_expand_next(len(keys), _p(keys), _p(merit), kcap, radius, W, room, _p(out))
    return out[:n]

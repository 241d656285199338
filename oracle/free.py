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
# the same source built twice: fixed step, and optimised timing (-DFREE_TIMED: the interval
# duration h is a fifth control, u = (F_n, F_t, v_x, v_y, h), two duration-bound rows)
_LIBS = {False: os.path.join(_HERE, "libfree_oracle.so"), True: os.path.join(_HERE, "libfree_timed_oracle.so")}

NX, NU, NW, NV, NE, NI, NR, NT = 5, 4, 9, 14, 8, 7, 15, 3
DIMS = {False: dict(NU=4, NW=9, NV=14, NI=7, NR=15), True: dict(NU=5, NW=10, NV=15, NI=9, NR=17)}
H_MIN, H_MAX, W_T = 0.02, 0.2, 0.01     # optimised timing: duration bounds, time charge
MAXSEG = 8
N_MODES = 16
N_TYPES = 16
# slider at rest at the origin, pusher 3 cm in front of face 3 (below the slider)
X0 = np.array([0.0, 0.0, 0.0, 0.0, -0.08])


def build(force: bool = False, timed: bool = False) -> str:
    out = _LIBS[timed]
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11", "-fPIC", "-shared",
             "-pthread"] + (["-DFREE_TIMED"] if timed else []) + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


_lib = {}


def lib(timed: bool = False):
    if timed not in _lib:
        from . import SolverParams
        L = C.CDLL(build(timed=timed))
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
        _lib[timed] = L
    return _lib[timed]


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
             nthreads=None, timed: bool = False):
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
    traj = np.zeros((B, nmax + 1, NX + DIMS[timed]["NU"]))
    stats = np.zeros((B, 4), np.int32)
    w = None if warm is None else _f64(warm)
    prm = params.c()
    rc = lib(timed).free_evaluate(B, smax, nmax, _p(x0), _p(goal), _p(inst), _p(nseg), _p(modes), _p(knots), _p(w),
                             C.byref(prm), nthreads or default_threads(), _p(cost), _p(viol), _p(feas), _p(traj),
                             _p(stats))
    if rc != 0:
        raise ValueError("free_evaluate rejected its arguments")
    return dict(cost=cost, viol=viol, feasible=feas, traj=traj, stats=stats)


def scales(timed: bool = False) -> np.ndarray:
    out = np.zeros(N_TYPES)
    lib(timed).free_scales(_p(out))
    return out


def rows(mode: int, mu: float, v, timed: bool = False):
    """Rows of one interval at v = (x_k, u_k, x_{k+1}) in physical units: (c, J, en, type)."""
    d = DIMS[timed]
    v = _f64(v)
    c, J = np.zeros(d["NR"]), np.zeros((d["NR"], d["NV"]))
    en, ty = np.zeros(d["NR"], np.int32), np.zeros(d["NR"], np.int32)
    if lib(timed).free_rows(int(mode), float(mu), _p(v), _p(c), _p(J), _p(en), _p(ty)) != 0:
        raise ValueError("bad mode")
    return c, J, en, ty


def cost(u, timed: bool = False):
    u = _f64(u)
    g = np.zeros(DIMS[timed]["NU"])
    return lib(timed).free_cost(_p(u), _p(g)), g


class Seq:
    """One order on one instance, for the pins (timed: the optimised-timing variant)."""

    def __init__(self, modes, knots, goal=(0.1, 0.1, np.pi / 4), mu=0.4, x0=X0, timed: bool = False):
        self.modes, self.knots = _i32(modes), _i32(knots)
        self.goal, self.mu, self.x0 = _f64(goal), float(mu), _f64(x0)
        self.N = int(self.knots.sum())
        self.timed = timed
        self.nu, self.nw = DIMS[timed]["NU"], DIMS[timed]["NW"]

    def initial(self):
        z = np.zeros(self.N * self.nw)
        n = lib(self.timed).free_initial(len(self.modes), _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal),
                                         self.mu, _p(z))
        if n < 0:
            raise ValueError("bad order")
        return z

    def score(self, z):
        J, v = C.c_double(), C.c_double()
        if lib(self.timed).free_score(len(self.modes), _p(self.modes), _p(self.knots), _p(self.x0), _p(self.goal),
                                      self.mu, _p(_f64(z)), C.byref(J), C.byref(v)) != 0:
            raise ValueError("bad order")
        return J.value, v.value

    def merit_grad_step(self, z, lam, nu, lamT, mu, rho):
        phi = C.c_double()
        g, dz = np.zeros(self.N * self.nw), np.zeros(self.N * self.nw)
        rc = lib(self.timed).free_merit_grad_step(len(self.modes), _p(self.modes), _p(self.knots), _p(self.x0),
                                                  _p(self.goal), self.mu, _p(_f64(z)), _p(_f64(lam)), _p(_f64(nu)),
                                                  _p(_f64(lamT)), float(mu), float(rho), C.byref(phi), _p(g), _p(dz))
        return phi.value, g, dz, rc == 0

    def args(self, z, k):
        """v = (x_k, u_k, x_{k+1}) of interval k"""
        z = _f64(z).reshape(self.N, self.nw)
        xk = self.x0 if k == 0 else z[k - 1, self.nu:]
        return np.concatenate([xk, z[k, :self.nu], z[k, self.nu:]])

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

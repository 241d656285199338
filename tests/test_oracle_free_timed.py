"""Pins of the free-motion pushing oracle with optimised timing (the paper's pushing
transcription, Sec. III-C and IV-A: the interval durations are controls with a duration
bound; the language of Sec. III-A).  The variant is the same C source built with
-DFREE_TIMED: u = (F_n, F_t, v_x, v_y, h), two duration-bound rows, a time charge w_T h in
the objective.  What pins it beyond its formulas: at h = dt every row is the fixed-step
free-motion row (pinned separately); central differences of rows, cost and merit; a dense
solve of the Gauss-Newton system; closed-form optima of a free approach followed by a
straight push with the durations free, inside and at both duration bounds.
"""
import itertools

import numpy as np
import pytest

from oracle import free as F

DT, HALF, HMIN, HMAX, WT = 0.1, 0.05, 0.02, 0.2, 0.01
# tight tolerances; stationarity 1e-9, since inside the duration bounds the optimum is a
# flat valley (see the closed form below) along which the gradient test converges slowly
TIGHT = dict(al_max=80, gn_max=40, eta_star=1e-12, omega_star=1e-9, rc_star=1e-12, mu_min=1e-8)


@pytest.fixture(scope="module")
def orc():
    import oracle
    F.build(timed=True)
    return oracle


def _timed_v(v14, h):
    return np.concatenate([v14[:9], [h], v14[9:]])


@pytest.mark.parametrize("mode", range(16))
def test_rows_at_the_fixed_step_are_the_free_motion_rows(orc, mode):
    """At h = dt every row and every Jacobian entry outside the h column equal the
    fixed-step model's; the duration rows read h_min - h and h - h_max."""
    rng = np.random.default_rng(700 + mode)
    scale = np.array([0.2, 0.2, 2, 0.06, 0.06, 2, 1, 0.1, 0.1, 0.2, 0.2, 2, 0.06, 0.06])
    for _ in range(4):
        v = rng.normal(size=14) * scale
        c0, J0, en0, ty0 = F.rows(mode, 0.37, v)
        c, J, en, ty = F.rows(mode, 0.37, _timed_v(v, DT), timed=True)
        assert np.array_equal(en[:15], en0) and np.array_equal(ty[:15], ty0)
        assert np.array_equal(c[:15], c0)
        assert np.array_equal(np.delete(J[:15], 9, axis=1), J0)
        assert en[15] == en[16] == 1 and c[15] == HMIN - DT and c[16] == DT - HMAX
        assert J[15, 9] == -1.0 and J[16, 9] == 1.0 and not np.any(np.delete(J[15:], 9, axis=1))


@pytest.mark.parametrize("mode", range(16))
def test_row_jacobians_match_central_differences(orc, mode):
    rng = np.random.default_rng(800 + mode)
    scale = np.array([0.2, 0.2, 2, 0.06, 0.06, 2, 1, 0.1, 0.1, 0.05, 0.2, 0.2, 2, 0.06, 0.06])
    for _ in range(4):
        v = rng.normal(size=15) * scale
        v[9] = abs(v[9]) + 0.02
        c, J, en, _ = F.rows(mode, 0.37, v, timed=True)
        Jfd = np.zeros_like(J)
        for j in range(15):
            h = 1e-6 * max(1.0, abs(v[j]))
            vp, vm = v.copy(), v.copy()
            vp[j] += h
            vm[j] -= h
            Jfd[:, j] = (F.rows(mode, 0.37, vp, timed=True)[0] - F.rows(mode, 0.37, vm, timed=True)[0]) / (2 * h)
        on = en.astype(bool)
        assert np.allclose(J[on], Jfd[on], rtol=1e-6, atol=1e-8)
        assert not np.any(J[~on]) and not np.any(c[~on])


def test_cost_gradient_and_scales(orc):
    fm = 0.5 * 9.81
    u = np.array([1.3, -0.4, 0.2, -0.7, 0.07])
    q = (u[0] ** 2 + u[1] ** 2) / fm ** 2 + u[2] ** 2 + u[3] ** 2 + WT
    J, g = F.cost(u, timed=True)
    assert abs(J - u[4] * q) <= 1e-16
    gfd = np.array([(F.cost(u + e, timed=True)[0] - F.cost(u - e, timed=True)[0]) / 2e-7
                    for e in 1e-7 * np.eye(5)])
    assert np.allclose(g, gfd, rtol=1e-7) and abs(g[4] - q) <= 1e-15
    s, s0 = F.scales(timed=True), F.scales()
    for t in (5, 6, 8, 9, 11, 12, 13, 14, 15):   # unit rows, the duration rows among them (type 13)
        assert s[t] == 1.0, t
    assert s[7] == s0[7] and s[10] == s0[10]     # rows without a duration column keep their scale
    assert np.all(s[:5] > s0[:5] - 1e-15)         # the defects gain the duration column


def _random_point(seed, modes=(15, 9, 15, 12, 0), knots=(3, 2, 3, 2, 2)):
    rng = np.random.default_rng(seed)
    S = F.Seq(modes, knots, goal=(0.08, 0.05, 0.4), mu=0.41, timed=True)
    z = S.initial() + 0.005 * rng.normal(size=S.N * S.nw)
    lam = 0.1 * rng.normal(size=S.N * F.NE)
    nu = np.abs(0.1 * rng.normal(size=S.N * F.DIMS[True]["NI"]))
    lamT = 0.1 * rng.normal(size=3)
    return S, z, lam, nu, lamT


def test_initial_guess_takes_the_fixed_step(orc):
    S = F.Seq([15, 9, 15, 12, 0], [3, 2, 3, 2, 2], timed=True)
    S0 = F.Seq([15, 9, 15, 12, 0], [3, 2, 3, 2, 2])
    z, z0 = S.initial().reshape(S.N, 10), S0.initial().reshape(S0.N, 9)
    assert np.all(z[:, 4] == DT) and np.array_equal(np.delete(z, 4, axis=1), z0)


@pytest.mark.parametrize("seed", [0, 1])
def test_merit_gradient_matches_central_differences(orc, seed):
    S, z, lam, nu, lamT = _random_point(seed)
    phi, g, _, _ = S.merit_grad_step(z, lam, nu, lamT, 0.05, 1e-3)
    gfd = np.zeros_like(g)
    for i in range(len(z)):
        zp, zm = z.copy(), z.copy()
        zp[i] += 1e-6
        zm[i] -= 1e-6
        gfd[i] = (S.merit_grad_step(zp, lam, nu, lamT, 0.05, 1e-3)[0] -
                  S.merit_grad_step(zm, lam, nu, lamT, 0.05, 1e-3)[0]) / 2e-6
    assert np.allclose(g, gfd, rtol=1e-5, atol=1e-7), np.abs(g - gfd).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_riccati_step_equals_dense_kkt_solve(orc, seed):
    """The backward Riccati recursion over the 10 stage unknowns gives the step of the dense
    system (H + rho I) dz = -g, H = sum over active scaled rows of a a^T / mu plus the cost
    Hessian model: 2 max(h, h_min / 2) on the force and velocity entries, none on h."""
    S, z, lam, nu, lamT = _random_point(seed)
    mu_al, rho, N, W, X, U = 0.03, 1e-3, S.N, S.nw, F.NX, S.nu
    NI, NR = F.DIMS[True]["NI"], F.DIMS[True]["NR"]
    _, g, dz, ok = S.merit_grad_step(z, lam, nu, lamT, mu_al, rho)
    assert ok
    sc = F.scales(timed=True)
    H = np.zeros((W * N, W * N))
    for k in range(N):
        c, J, en, ty = F.rows(S.mode_of(k), S.mu, S.args(z, k), timed=True)
        cols = ([(k - 1) * W + U + i for i in range(X)] if k > 0 else [None] * X) + [k * W + i for i in range(W)]
        for r in range(NR):
            if not en[r]:
                continue
            cs, a_row = c[r] / sc[ty[r]], J[r] / sc[ty[r]]
            if r >= F.NE and not (nu[k * NI + r - F.NE] + cs / mu_al > 0):
                continue
            a = np.zeros(W * N)
            for j, col in enumerate(cols):
                if col is not None:
                    a[col] += a_row[j]
            H += np.outer(a, a) / mu_al
        hm = max(z[k * W + 4], HMIN / 2)
        H[k * W:k * W + 2, k * W:k * W + 2] += np.eye(2) * hm * 2 / (0.5 * 9.81) ** 2
        H[k * W + 2:k * W + 4, k * W + 2:k * W + 4] += np.eye(2) * hm * 2
    for r in range(3):
        a = np.zeros(W * N)
        a[(N - 1) * W + U + r] = 1.0 / sc[14 if r < 2 else 15]
        H += np.outer(a, a) / mu_al
    dz_dense = np.linalg.solve(H + rho * np.eye(len(z)), -g)
    assert np.linalg.norm(dz - dz_dense) <= 1e-6 * np.linalg.norm(dz_dense)


def _solve(orc, modes, knots, goal, x0, params):
    m = np.zeros((1, 8), np.int32)
    k = np.zeros((1, 8), np.int32)
    m[0, :len(modes)], k[0, :len(knots)] = modes, knots
    return F.evaluate(np.array([x0]), np.array([goal]), np.array([0.4]), np.array([len(modes)]), m, k, params,
                      timed=True)


def _segment_cost(D, N):
    """least sum_k h_k (q_k + w_T) for a move of length D in N steps, q = (D / (N h))^2 per
    unit weight and h in [h_min, h_max]: h* = D / (N sqrt(w_T)) clipped, constant"""
    h = min(max(D / (N * np.sqrt(WT)), HMIN), HMAX)
    return D ** 2 / (N * h) + N * h * WT, h


@pytest.mark.parametrize("d,N1,N2", [(0.05, 6, 10), (0.12, 10, 12), (0.02, 4, 6), (0.3, 6, 10), (0.005, 4, 10)])
def test_free_approach_then_straight_push_closed_form(orc, d, N1, N2):
    """Pusher 3 cm in front of face 2, goal (d, 0, 0), order [free in front of face 2,
    stick on face 2] with the durations free: the approach costs sum h (|v|^2 + w_T) for a
    3 cm move, the push sum h (F_n^2 / f_max^2 + w_T) for a slider move of d (the limit
    surface gives dx = h F_n / f_max per step, v_ref = 1 m/s); each is least at
    2 D sqrt(w_T) when D / (N sqrt(w_T)) lies inside [h_min, h_max], else with every duration
    at the bound it passes (D^2 / (N h) + N h w_T).  Cases inside the bounds, at h_max
    (d = 0.3) and at h_min (d = 0.005)."""
    x0 = np.array([0.0, 0.0, 0.0, -0.08, 0.0])
    J1, h1 = _segment_cost(0.03, N1)
    J2, h2 = _segment_cost(d, N2)
    Jstar = J1 + J2
    r = _solve(orc, [F.free(2), F.contact(2, 0)], [N1, N2], (d, 0.0, 0.0), x0, orc.Params(**TIGHT))
    assert r["feasible"][0] == 1 and r["stats"][0, 3] == 1
    assert abs(r["cost"][0] - Jstar) <= 1e-6 * Jstar, (r["cost"][0], Jstar)
    T = r["traj"][0]
    # inside the bounds the optimum is not unique (cost 2 sqrt(w_T) sum |s_k| for steps s_k):
    # any split of the move at speed sqrt(w_T), so the segment lasts D / sqrt(w_T); at a
    # bound every duration sits on it
    for D, sl, h in ((0.03, slice(0, N1), h1), (d, slice(N1, N1 + N2), h2)):
        if HMIN < h < HMAX:
            assert abs(T[sl, 9].sum() - D / np.sqrt(WT)) <= 1e-4 * D / np.sqrt(WT), (T[sl, 9], D)
            assert np.all(T[sl, 9] >= HMIN - 1e-7) and np.all(T[sl, 9] <= HMAX + 1e-7)
        else:
            assert np.allclose(T[sl, 9], h, rtol=1e-4), (T[sl, 9], h)
    assert np.allclose(T[N1, 3:5], [-HALF, 0.0], atol=1e-6)


def test_language_is_the_fixed_step_one(orc):
    """Keys, seed and neighbourhoods do not depend on the timing (one language)."""
    assert np.array_equal(F.seed(5), F.seed(5))
    for o in itertools.islice(itertools.product(range(16), repeat=3), 0, 4096, 37):
        assert F.admissible(o) == bool(F.lib(True).free_admissible(3, F._i32(list(o)).ctypes.data_as(F.C.c_void_p)))

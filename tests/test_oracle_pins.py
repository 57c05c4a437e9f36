"""Pins of the FP64 CPU reference against facts fixed outside it.

Each test checks the reference against something it does not compute itself:
published known-answer vectors, closed forms of the RK4 map on linear
dynamics, an independent high-accuracy ODE solver, exact affine ratio tests,
brute-force grids and invariants of the method (recursive feasibility,
monotonicity in N and H, v = r when r is admissible).
"""
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2510_08288_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# Random numbers
# ----------------------------------------------------------------------------

def test_philox_known_answers(oracle_mod):
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = oracle_mod.philox(r[0:4], r[4:6])
        assert [int(v) for v in out] == r[6:10]


def test_uniform_box_edges_and_grid(oracle_mod):
    # u = (word >> 8) 2^-24 spans [0, 1) on a grid of 2^-24; lo maps to fl32(lo).
    lo, hi = -0.05, 0.05
    assert oracle_mod.uniform_box(0, lo, hi) == np.float32(lo)
    top = oracle_mod.uniform_box(0xFFFFFFFF, lo, hi)
    assert np.float32(lo) < top < np.float32(hi)
    # word and word + 255 share the same top 24 bits -> same value
    assert oracle_mod.uniform_box(0x12345600, lo, hi) == oracle_mod.uniform_box(0x123456FF, lo, hi)
    # exact value for a representable case: span 1, lo 0
    assert oracle_mod.uniform_box(0x80000000, 0.0, 1.0) == 0.5


def test_draw_statistics(oracle_mod):
    # Moments and Kolmogorov-Smirnov distance of the scenario draws against U[lo, hi).
    p = W.lq4_problem(N=64, H=10)
    o = oracle_mod.Oracle(p)
    vals = np.array([o.draw_w(3, k, j) for k in range(400) for j in range(25)])
    n = vals.shape[0]
    for c in range(2):
        x = (vals[:, c] + 0.05) / 0.1
        assert abs(x.mean() - 0.5) < 4 * np.sqrt(1 / 12 / n)
        assert abs(x.var() - 1 / 12) < 4 * np.sqrt(1 / 180 / n)
        xs = np.sort(x)
        ks = np.max(np.maximum(np.arange(1, n + 1) / n - xs, xs - np.arange(n) / n))
        assert ks < 1.63 / np.sqrt(n)  # 1% critical value
    # independence of the two components and of consecutive steps
    assert abs(np.corrcoef(vals[:, 0], vals[:, 1])[0, 1]) < 4 / np.sqrt(n)
    # fresh draws per RG step t, shared across candidates (common random numbers)
    assert not np.array_equal(o.draw_w(3, 5, 7), o.draw_w(4, 5, 7))
    assert np.array_equal(o.draw_w(3, 5, 7), o.draw_w(3, 5, 7))


def test_theta_draws_relative_box(oracle_mod):
    p = W.fc9_problem(N=16, H=10)
    o = oracle_mod.Oracle(p)
    nom = W.FC9_THETA_NOM
    ths = np.array([o.draw_theta(0, k) for k in range(500)])
    ratio = ths / nom[None, :]
    assert ratio.min() >= 0.9 - 1e-7 and ratio.max() < 1.1 + 1e-7
    assert abs(ratio.mean() - 1.0) < 0.01


# ----------------------------------------------------------------------------
# RK4 on linear dynamics: the matrix-polynomial closed form
# ----------------------------------------------------------------------------

def _lq4_mats(p):
    c = p.coeffs
    A = c[0:16].reshape(4, 4)
    B = c[16:20]
    G = c[20:36].reshape(4, 4)
    E = c[36:44].reshape(4, 2)
    C = c[44:52].reshape(2, 4)
    return A, B, G, E, C


def _rk4_poly(A, h):
    Z = h * A
    I = np.eye(A.shape[0])
    Z2 = Z @ Z
    Z3 = Z2 @ Z
    Z4 = Z3 @ Z
    Phi = I + Z + Z2 / 2 + Z3 / 6 + Z4 / 24
    Psi = h * (I + Z / 2 + Z2 / 6 + Z3 / 24)   # input map of a constant forcing
    return Phi, Psi


def _linear_problem(seed=3, **kw):
    p = W.lq4_problem(seed=seed, quad_scale=0.0, **kw)
    return p


@pytest.mark.parametrize("inject", [W.INJECT_ODE, W.INJECT_POST])
def test_rk4_closed_form_linear(oracle_mod, inject):
    p = _linear_problem(N=4, H=300, dt=0.01, inject=inject)
    o = oracle_mod.Oracle(p)
    A, B, _, E, _ = _lq4_mats(p)
    Phi, Psi = _rk4_poly(A, p.dt)
    rng = np.random.default_rng(0)
    x0 = rng.uniform(-0.3, 0.3, 4)
    v, t, k = 0.7, 5, 2
    _, _, _, traj = o.rollout(x0, v, t, k, traj=True)
    x = x0.copy()
    for j in range(p.H):
        w = o.draw_w(t, k, j)
        if inject == W.INJECT_ODE:
            x = Phi @ x + Psi @ (B * v + E @ w)
        else:
            x = Phi @ x + Psi @ (B * v) + E @ w
        np.testing.assert_allclose(traj[j + 1], x, rtol=1e-12, atol=1e-13)


def test_rk4_matrix_powers_zero_disturbance(oracle_mod):
    # x_j = Phi^j x0 + sum_{i<j} Phi^i Gamma v  (zero-width disturbance box)
    p = _linear_problem(N=1, H=500, dt=0.01, w_half=0.0)
    o = oracle_mod.Oracle(p)
    A, B, _, _, _ = _lq4_mats(p)
    Phi, Psi = _rk4_poly(A, p.dt)
    Gam = Psi @ B
    x0 = np.array([0.1, -0.2, 0.05, 0.3])
    v = -1.3
    _, _, _, traj = o.rollout(x0, v, 0, 0, traj=True)
    for j in [1, 7, 100, 500]:
        Pj = np.linalg.matrix_power(Phi, j)
        S = sum(np.linalg.matrix_power(Phi, i) for i in range(j))
        np.testing.assert_allclose(traj[j], Pj @ x0 + S @ Gam * v, rtol=1e-11, atol=1e-13)


def test_rk4_fourth_order_quadratic_plant(oracle_mod):
    # Nonlinear LQ4 (G != 0): global error of the oracle's RK4 against a
    # high-accuracy integration of xdot = A x + B v + G x^2 shrinks ~16x per halving.
    p = W.lq4_problem(seed=5, N=1, H=10, w_half=0.0, quad_scale=0.2)
    A, B, G, _, _ = _lq4_mats(p)
    v = 1.1
    x0 = np.array([0.4, -0.3, 0.2, 0.1])
    Tf = 1.0
    ref = solve_ivp(lambda _t, x: A @ x + B * v + G @ (x * x), (0, Tf), x0,
                    method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
    errs = []
    for h in [0.1, 0.05, 0.025]:
        q = p.replace(dt=h, H=int(round(Tf / h)))
        _, _, _, traj = oracle_mod.Oracle(q).rollout(x0, v, 0, 0, traj=True)
        errs.append(np.max(np.abs(traj[-1] - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def _fc9_rhs_def(coeffs, theta, x, v, w):
    """FC9 dynamics written from the plant definition (for the solver pin)."""
    Wm = coeffs[:81].reshape(9, 9)
    xbar = coeffs[81:90]
    c_q0, p_amb, _, _, p1ref = coeffs[110:115]
    a, kq, b, mu = theta[:9], theta[9:15], theta[15:18], theta[18:20]
    z = x - xbar
    p = np.append(x[:6], p_amb)
    q = np.concatenate([[c_q0 * x[6]], kq * np.sqrt(np.maximum(p[:6] - p[1:7], 0.0))])
    phi = np.zeros(9)
    phi[:6] = q[:6] - q[1:7]
    phi[6] = b[0] * v - mu[0] * x[6] * (x[0] - p1ref)
    phi[7] = b[1] * v * x[6]
    phi[8] = b[2] * v - mu[1] * (x[8] - 1.0) * v
    return -a * z + Wm @ np.tanh(z) + w + phi


def test_fc9_rk4_fourth_order(oracle_mod):
    p = W.fc9_problem(N=1, H=10, w_half=0.0)
    o = oracle_mod.Oracle(p)
    theta = o.draw_theta(0, 0)
    v = 1.0
    x0 = W.FC9_XBAR + 0.05 * np.arange(9) / 9.0
    # pressures decrease along the chain so every orifice stays open
    wv = np.zeros(9)
    np.testing.assert_allclose(o.rhs(x0, v, wv, theta), _fc9_rhs_def(p.coeffs, theta, x0, v, wv),
                               rtol=1e-14, atol=1e-14)
    Tf = 0.5
    ref = solve_ivp(lambda _t, x: _fc9_rhs_def(p.coeffs, theta, x, v, wv), (0, Tf), x0,
                    method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
    errs = []
    for h in [0.02, 0.01, 0.005]:   # h * |a9| well inside the asymptotic range
        q = p.replace(dt=h, H=int(round(Tf / h)))
        oq = oracle_mod.Oracle(q)
        x = x0.copy()
        for _ in range(q.H):
            x = oq.step(x, v, wv, theta)
        errs.append(np.max(np.abs(x - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


# ----------------------------------------------------------------------------
# Margins and the steady-state test
# ----------------------------------------------------------------------------

def test_box_margin_is_one_minus_max_abs(oracle_mod):
    p = W.lq4_problem()
    o = oracle_mod.Oracle(p)
    rng = np.random.default_rng(1)
    for _ in range(200):
        y = rng.normal(0, 1.5, 2)
        assert o.margin(y) == pytest.approx(1.0 - np.max(np.abs(y)), abs=1e-15)
    assert o.margin(np.array([np.nan, 0.0])) == -np.inf


def test_steady_state_linear_is_dc_gain(oracle_mod):
    # G = 0: y_ss = H0 v with H0 = -C A^{-1} B, the fixed point of the RK4 map too.
    p = _linear_problem(N=1, H=10)
    o = oracle_mod.Oracle(p)
    A, B, _, _, C = _lq4_mats(p)
    Phi, Psi = _rk4_poly(A, p.dt)
    for v in [-1.7, 0.3, 2.0]:
        m, xs, _ = o.steady_margin(v)
        np.testing.assert_allclose(xs, -np.linalg.solve(A, B) * v, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(xs, np.linalg.solve(np.eye(4) - Phi, Psi @ B) * v,
                                   rtol=1e-9, atol=1e-12)
        y = C @ xs
        assert m == pytest.approx((1 - p.eps) - np.max(np.abs(y)), abs=1e-13)


def test_steady_state_quadratic_residual_and_convergence(oracle_mod):
    # G != 0: Newton's equilibrium solves A x + B v + G x^2 = 0 and a long
    # disturbance-free rollout settles on it.
    p = W.lq4_problem(seed=7, N=1, H=4000, dt=0.01, w_half=0.0)
    o = oracle_mod.Oracle(p)
    A, B, G, _, C = _lq4_mats(p)
    for v in [-1.0, 0.5, 1.5]:
        m, xs, it = o.steady_margin(v)
        assert np.max(np.abs(A @ xs + B * v + G @ (xs * xs))) < 1e-12
        _, _, _, traj = o.rollout(np.zeros(4), v, 0, 0, traj=True)
        np.testing.assert_allclose(traj[-1], xs, atol=1e-9)


def test_fc9_equilibrium(oracle_mod):
    p = W.fc9_problem(N=1, H=20000, dt=0.002, w_half=0.0)
    o = oracle_mod.Oracle(p)
    for v in [0.5, 1.0]:
        m, xs, it = o.steady_margin(v)
        assert np.isfinite(m)
        res = _fc9_rhs_def(p.coeffs, W.FC9_THETA_NOM, xs, v, np.zeros(9))
        assert np.max(np.abs(res)) < 1e-12
        # integrate the nominal model (nominal theta: zero relative spread)
        q = p.replace(theta_rel=0.0)
        oq = oracle_mod.Oracle(q)
        _, _, _, traj = oq.rollout(W.FC9_XBAR, v, 0, 0, traj=True)
        np.testing.assert_allclose(traj[-1], xs, atol=1e-7)


def test_nonfinite_rollout_is_infeasible(oracle_mod):
    # A strongly destabilising quadratic term blows the state up: margin -inf.
    p = W.lq4_problem(seed=7, N=2, H=3000, dt=0.01, quad_scale=3.0)
    o = oracle_mod.Oracle(p)
    m, j, _ = o.rollout(np.zeros(4), 2.0, 0, 0)
    assert m == -np.inf or m < -1e6


# ----------------------------------------------------------------------------
# Searches
# ----------------------------------------------------------------------------

def _affine_kappa_star(o, p, x0, r, v_prev, t):
    """Linear plant with fixed draws: every margin row is affine in kappa, so the
    largest admissible kappa is a ratio test (x_j(v) = x_j(0) + v dx_j)."""
    A, B, _, E, C = _lq4_mats(p)
    Phi, Psi = _rk4_poly(A, p.dt)
    F, g = p.F, p.g
    lo_a, rows = [], []
    va, vb = v_prev, r          # v(kappa) = v_prev + kappa (r - v_prev)
    kstar = 1.0
    for k in range(p.N):
        xa = x0.copy()
        xb = x0.copy()
        for j in range(p.H + 1):
            ma = g - F @ (C @ xa)
            mb = g - F @ (C @ xb)
            a, b = ma, mb - ma       # margin(kappa) = a + b kappa
            assert np.all(a >= 0)
            for ai, bi in zip(a, b):
                if bi < 0:
                    kstar = min(kstar, -ai / bi)
            if j == p.H:
                break
            w = o.draw_w(t, k, j)
            xa = Phi @ xa + Psi @ (B * va + E @ w)
            xb = Phi @ xb + Psi @ (B * vb + E @ w)
    H0 = -C @ np.linalg.solve(A, B)
    gt = g - p.eps * np.abs(g)
    a = gt - F @ (H0 * va)
    b = gt - F @ (H0 * vb) - a
    for ai, bi in zip(a, b):
        if bi < 0:
            kstar = min(kstar, -ai / bi)
    return kstar


@pytest.mark.parametrize("seed,r", [(3, 1.5), (4, -2.0), (6, 2.5), (8, 1.0), (9, -1.2)])
def test_bisection_exact_linear_ratio(oracle_mod, seed, r):
    p = _linear_problem(seed=seed, N=6, H=150, dt=0.01)
    o = oracle_mod.Oracle(p)
    x0 = np.zeros(4)
    K = 12
    ks = _affine_kappa_star(o, p, x0, r, 0.0, 0)
    res = o.bisect(x0, r, 0.0, 0, K)
    if ks >= 1.0:
        assert res["kappa"] == 1.0 and res["passes"] == 1 and res["v"] == r
    else:
        scaled = ks * 2 ** K
        if abs(scaled - round(scaled)) < 1e-9:
            pytest.skip("kappa* too close to a dyadic point")
        assert res["kappa"] == np.floor(scaled) / 2 ** K
        assert res["passes"] == K + 1


def _verdicts(o, x0, r, v_prev, t, kappas):
    return np.array([o.candidate(x0, o.candidate_v(k, r, v_prev), t)[0] >= 0 for k in kappas])


@pytest.mark.parametrize("seed", [7, 12, 21])
def test_bisection_matches_brute_force_grid(oracle_mod, seed):
    p = W.lq4_problem(seed=seed, N=8, H=100, dt=0.01)
    o = oracle_mod.Oracle(p)
    x0 = np.zeros(4)
    K = 6
    r = 1.5
    grid = np.arange(2 ** K + 1) / 2 ** K
    ok = _verdicts(o, x0, r, 0.0, 0, grid)
    res = o.bisect(x0, r, 0.0, 0, K)
    kb = res["kappa"]
    # bracket invariant: the result is admissible (or 0), the next dyadic is not (or 1)
    ib = int(round(kb * 2 ** K))
    assert kb == ib / 2 ** K
    if ib > 0:
        assert ok[ib]
    if ib < 2 ** K:
        assert not ok[ib + 1]
    # monotone pattern (admissible prefix): bisection returns the largest admissible dyadic
    first_bad = np.argmin(ok) if not ok.all() else len(ok)
    if ok[:first_bad].all() and not ok[first_bad:].any():
        assert ib == first_bad - 1 if first_bad > 0 else ib == 0


def test_bisection_trace_follows_alg1(oracle_mod):
    wl = W.workload_lq4_fp64_single()
    o = oracle_mod.Oracle(wl["problem"])
    res = o.bisect(wl["x0"], wl["r"], wl["v_prev"], 0, 12, trace=True)
    tk, tm = res["trace_kappa"], res["trace_margin"]
    assert tk[0] == 1.0
    lo, hi = 0.0, 1.0
    for i in range(1, len(tk)):
        if tm[i - 1] >= 0:
            lo = tk[i - 1]
        else:
            hi = tk[i - 1]
        assert tk[i] == (lo + hi) / 2
    assert res["kappa"] == (lo if tm[-1] < 0 else tk[-1])


def test_v_equals_r_when_admissible(oracle_mod):
    p = W.lq4_problem(seed=7, N=16, H=200)
    o = oracle_mod.Oracle(p)
    for r in [0.05, -0.1, 0.2]:
        res = o.bisect(np.zeros(4), r, 0.0, 0, 12)
        assert res["kappa"] == 1.0 and res["v"] == r and res["passes"] == 1


def test_alg1_equals_alg2_single_scenario_no_disturbance(oracle_mod):
    p = W.lq4_problem(seed=7, N=1, H=200, w_half=0.0)
    o = oracle_mod.Oracle(p)
    for r in [1.5, -2.0, 0.9]:
        a = o.bisect(np.zeros(4), r, 0.0, 0, 12)
        b = o.alg2(np.zeros(4), r, 0.0, 0, 12)
        assert a["kappa"] == b["kappa"]


def test_alg2_equals_joint_bisection_monotone(oracle_mod):
    p = W.lq4_problem(seed=7, N=6, H=120)
    o = oracle_mod.Oracle(p)
    x0 = np.zeros(4)
    K = 8
    grid = np.arange(2 ** K + 1) / 2 ** K
    for r in [1.5, -1.8]:
        # per-scenario monotonicity on the dyadic grid makes the two forms equal
        a = o.bisect(x0, r, 0.0, 0, K)
        b = o.alg2(x0, r, 0.0, 0, K)
        ok = _verdicts(o, x0, r, 0.0, 0, grid)
        fb = np.argmin(ok) if not ok.all() else len(ok)
        if ok[:fb].all() and not ok[fb:].any():
            assert a["kappa"] == b["kappa"]


def test_grid_alg3_and_dyadic_grid_equivalence(oracle_mod):
    p = W.lq4_problem(seed=7, N=8, H=120)
    o = oracle_mod.Oracle(p)
    x0 = np.zeros(4)
    K = 5
    M = 2 ** K + 1
    res = o.grid(x0, 1.5, 0.0, 0, M, 0, want_P=True)
    P = res["P"]
    rows = np.where(P.all(axis=1))[0]
    assert res["kappa"] == (rows.max() / (M - 1) if len(rows) else 0.0)
    ok = P.all(axis=1)
    fb = np.argmin(ok) if not ok.all() else len(ok)
    if ok[:fb].all() and not ok[fb:].any():
        assert o.bisect(x0, 1.5, 0.0, 0, K)["kappa"] == res["kappa"]


def test_grid_refinement_brackets(oracle_mod):
    p = W.lq4_problem(seed=7, N=8, H=120)
    o = oracle_mod.Oracle(p)
    x0 = np.zeros(4)
    M, ref = 16, 5
    res = o.grid(x0, 1.5, 0.0, 0, M, ref)
    plain = o.grid(x0, 1.5, 0.0, 0, M, 0)
    k = res["kappa"]
    assert plain["kappa"] <= k < plain["kappa"] + 1.0 / (M - 1)
    v = o.candidate_v(k, 1.5, 0.0)
    assert o.candidate(x0, v, 0)[0] >= 0
    step = (1.0 / (M - 1)) / 2 ** ref
    assert o.candidate(x0, o.candidate_v(k + step * 1.0000001, 1.5, 0.0), 0)[0] < 0 or k + step >= 1


def test_monotone_in_scenarios_and_horizon(oracle_mod):
    # Counter-based draws: the first N1 scenarios (and H1 steps) are a prefix of
    # the larger set, so the admissible set can only shrink.
    x0 = np.zeros(4)
    ks = []
    for N in [1, 4, 16, 64]:
        p = W.lq4_problem(seed=7, N=N, H=200)
        ks.append(oracle_mod.Oracle(p).bisect(x0, 1.5, 0.0, 0, 10)["kappa"])
    assert all(a >= b for a, b in zip(ks, ks[1:]))
    kh = []
    for H in [20, 60, 200, 400]:
        p = W.lq4_problem(seed=7, N=16, H=H)
        kh.append(oracle_mod.Oracle(p).bisect(x0, 1.5, 0.0, 0, 10)["kappa"])
    assert all(a >= b for a, b in zip(kh, kh[1:]))


def test_zero_width_box_equals_single_scenario(oracle_mod):
    x0 = np.zeros(4)
    p1 = W.lq4_problem(seed=7, N=1, H=200, w_half=0.0)
    p64 = W.lq4_problem(seed=7, N=64, H=200, w_half=0.0)
    a = oracle_mod.Oracle(p1).bisect(x0, 1.5, 0.0, 0, 12)
    b = oracle_mod.Oracle(p64).bisect(x0, 1.5, 0.0, 0, 12)
    assert a["kappa"] == b["kappa"]


def test_thread_count_does_not_change_results(oracle_mod):
    p = W.lq4_problem(seed=7, N=37, H=150)
    x0 = np.zeros(4)
    a = oracle_mod.Oracle(p, nthreads=1).candidate(x0, 0.8, 2)
    b = oracle_mod.Oracle(p, nthreads=5).candidate(x0, 0.8, 2)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and a[2] == b[2]


# ----------------------------------------------------------------------------
# Closed loop
# ----------------------------------------------------------------------------

def test_recursive_feasibility_without_disturbance(oracle_mod):
    # True plant = model and no disturbance: the previous prediction's tail is
    # the new prediction, so kappa = 0 stays admissible at every step.
    p = W.lq4_problem(seed=7, N=2, H=600, dt=0.01, w_half=0.0)
    o = oracle_mod.Oracle(p)
    r_seq = W.reference_sequence(5, 40, switch_every=10, lo=-2, hi=2)
    out = o.closed_loop(np.zeros(4), 0.0, r_seq, K=10)
    v_prev = 0.0
    for s in range(len(r_seq)):
        M0 = o.candidate(out["x"][s], v_prev, s)[0]
        assert M0 >= 0
        v_prev = out["v"][s]
    # outputs stay inside the box along the realised trajectory
    A, B, G, E, C = _lq4_mats(p)
    assert np.all(np.abs(out["x"] @ C.T) <= 1 + 1e-12)


def test_closed_loop_resume_is_exact(oracle_mod):
    p = W.lq4_problem(seed=7, N=8, H=150)
    o = oracle_mod.Oracle(p)
    r_seq = W.reference_sequence(5, 12, switch_every=4)
    full = o.closed_loop(np.zeros(4), 0.0, r_seq, K=8)
    a = o.closed_loop(np.zeros(4), 0.0, r_seq[:5], K=8)
    b = o.closed_loop(a["x"][-1], a["v"][-1], r_seq[5:], t0=5, K=8)
    assert np.array_equal(full["v"], np.concatenate([a["v"], b["v"]]))


# ----------------------------------------------------------------------------
# Sensitivities (forward-mode tangents) against finite differences and the
# linear closed form
# ----------------------------------------------------------------------------

def test_tangent_linear_closed_form(oracle_mod):
    # G = 0, w fixed: x_j(v) = x_j(0) + v * sum_{i<j} Phi^i Psi B, so
    # dm/dv = -F_r* C sum_{i<j*} Phi^i Psi B exactly.
    p = _linear_problem(seed=3, N=4, H=300, dt=0.01)
    o = oracle_mod.Oracle(p)
    A, B, _, _, C = _lq4_mats(p)
    Phi, Psi = _rk4_poly(A, p.dt)
    x0 = np.array([0.1, 0.0, -0.1, 0.05])
    for v in [0.4, -0.7]:
        for k in range(3):
            m, dv, _, j, r = o.rollout_tangent(x0, v, 2, k)
            S = sum(np.linalg.matrix_power(Phi, i) for i in range(j)) @ Psi @ B if j > 0 else np.zeros(4)
            ref = -(p.F[r] @ C @ S)
            assert dv == pytest.approx(ref, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("kind", ["lq4", "fc9"])
def test_tangent_matches_central_differences(oracle_mod, kind):
    if kind == "lq4":
        p = W.lq4_problem(seed=24, N=4, H=400, dt=0.005, eps=0.01)
        x0 = np.zeros(4)
        vs = [0.6, -0.9]
    else:
        p = W.fc9_problem(N=4, H=400, dt=0.002)
        o0 = oracle_mod.Oracle(p)
        x0 = o0.steady_margin(0.5)[1]
        vs = [1.1, 1.4]
    o = oracle_mod.Oracle(p)
    h = 1e-4
    checked = 0
    for v in vs:
        for k in range(p.N):
            m, dv, dth, j, r = o.rollout_tangent(x0, v, 0, k)
            mp, jp, rp = o.rollout(x0, v + h, 0, k)
            mm, jm, rm = o.rollout(x0, v - h, 0, k)
            if (jp, rp) != (j, r) or (jm, rm) != (j, r):
                continue   # minimiser moves inside the stencil: not differentiable there
            fd = (mp - mm) / (2 * h)
            assert dv == pytest.approx(fd, rel=1e-6, abs=1e-9)
            checked += 1
            for q in range(p.n_theta):
                cp = p.coeffs.copy(); cp[90 + q] += h * p.coeffs[90 + q]
                cm = p.coeffs.copy(); cm[90 + q] -= h * p.coeffs[90 + q]
                op = oracle_mod.Oracle(p.replace(coeffs=cp))
                om = oracle_mod.Oracle(p.replace(coeffs=cm))
                a, ja_, ra_ = op.rollout(x0, v, 0, k)
                b, jb_, rb_ = om.rollout(x0, v, 0, k)
                if (ja_, ra_) != (j, r) or (jb_, rb_) != (j, r):
                    continue
                fdq = (a - b) / (2 * h * p.coeffs[90 + q])
                assert dth[q] == pytest.approx(fdq, rel=1e-5, abs=1e-8), q
    assert checked >= 2


def test_steady_tangent_matches_central_differences(oracle_mod):
    for p, vs in [(W.lq4_problem(seed=24, N=1, H=10, eps=0.01), [0.3, -0.6]),
                  (W.fc9_problem(N=1, H=10), [0.8, 1.3])]:
        o = oracle_mod.Oracle(p)
        h = 1e-5
        for v in vs:
            m, dv, dth = o.steady_tangent(v)
            fd = (o.steady_margin(v + h)[0] - o.steady_margin(v - h)[0]) / (2 * h)
            assert dv == pytest.approx(fd, rel=1e-6, abs=1e-9)
            for q in range(p.n_theta):
                cp = p.coeffs.copy(); cp[90 + q] += h
                cm = p.coeffs.copy(); cm[90 + q] -= h
                fdq = (oracle_mod.Oracle(p.replace(coeffs=cp)).steady_margin(v)[0]
                       - oracle_mod.Oracle(p.replace(coeffs=cm)).steady_margin(v)[0]) / (2 * h)
                assert dth[q] == pytest.approx(fdq, rel=1e-5, abs=1e-8)


def test_candidate_grad_matches_kappa_differences(oracle_mod):
    p = W.lq4_problem(seed=24, N=16, H=500, dt=0.005, eps=0.01)
    o = oracle_mod.Oracle(p)
    x0 = np.zeros(4)
    h = 1e-5
    for kap in [0.3, 0.45]:
        M, dk, _, ka = o.candidate_grad(x0, kap, 1.8, 0.0, 0)
        Mp, _, _, kp = o.candidate_grad(x0, kap + h, 1.8, 0.0, 0)
        Mm, _, _, km = o.candidate_grad(x0, kap - h, 1.8, 0.0, 0)
        if kp == ka == km:
            assert dk == pytest.approx((Mp - Mm) / (2 * h), rel=1e-5, abs=1e-8)


# ----------------------------------------------------------------------------
# Safeguarded Newton search
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed,r", [(3, 1.5), (4, -2.0), (6, 2.5), (8, 1.0)])
def test_newton_exact_linear_ratio(oracle_mod, seed, r):
    # The linear plant's exact kappa*: Newton must stop within 2^-K below it.
    p = _linear_problem(seed=seed, N=6, H=150, dt=0.01)
    o = oracle_mod.Oracle(p)
    K = 12
    ks = _affine_kappa_star(o, p, np.zeros(4), r, 0.0, 0)
    res = o.newton(np.zeros(4), r, 0.0, 0, K)
    if ks >= 1.0:
        assert res["kappa"] == 1.0
    else:
        assert ks - 2.0 ** -K - 1e-12 <= res["kappa"] <= ks + 1e-12
    assert res["rounds"] <= K + 2


@pytest.mark.parametrize("seed,r", [(24, 1.5), (24, -1.8), (10, 1.9), (19, -1.5), (7, 1.5)])
def test_newton_agrees_with_bisection(oracle_mod, seed, r):
    p = W.lq4_problem(seed=seed, N=16, H=600, dt=0.005, eps=0.01)
    o = oracle_mod.Oracle(p, nthreads=4)
    b = o.bisect(np.zeros(4), r, 0.0, 0, 12)
    n = o.newton(np.zeros(4), r, 0.0, 0, 12)
    assert abs(n["kappa"] - b["kappa"]) <= 2.0 ** -12
    if n["kappa"] > 0:
        assert o.candidate(np.zeros(4), o.candidate_v(n["kappa"], r, 0.0), 0)[0] >= 0


def test_newton_fc9_bracket(oracle_mod):
    p = W.fc9_problem(N=16, H=300, dt=0.002)
    o = oracle_mod.Oracle(p, nthreads=4)
    x0 = o.steady_margin(0.5)[1]
    n = o.newton(x0, 2.0, 0.5, 0, 12)
    b = o.bisect(x0, 2.0, 0.5, 0, 12)
    assert 0 < n["kappa"] < 1
    assert abs(n["kappa"] - b["kappa"]) <= 2.0 ** -12
    assert o.candidate(x0, o.candidate_v(n["kappa"], 2.0, 0.5), 0)[0] >= 0
    assert o.candidate(x0, o.candidate_v(n["kappa"] + 2.0 ** -12, 2.0, 0.5), 0)[0] < 0


@pytest.mark.parametrize("vp,r", [(0.7954, 1.377), (-0.8452, -1.15)])
def test_newton_refused_everywhere_ends_in_two_rounds(oracle_mod, vp, r):
    # From the equilibrium of v_prev (admissible now) a wide disturbance box
    # refuses every candidate: both searches return kappa = 0 (status 1).
    # Newton's step lands below the admissible end, moves to lo + 2^-K, is
    # refused there and closes the bracket in the second round (bisection
    # needs all K + 1 evaluations).
    p = W.lq4_problem(seed=24, N=32, H=300, dt=0.005, eps=0.01, w_half=0.3)
    o = oracle_mod.Oracle(p, nthreads=4)
    x0 = o.steady_margin(vp)[1]
    b = o.bisect(x0, r, vp, 0, 12)
    assert b["status"] == 1 and b["kappa"] == 0.0 and b["passes"] == 13
    n = o.newton(x0, r, vp, 0, 12)
    assert n["status"] == 1 and n["kappa"] == 0.0
    assert n["rounds"] == 2 and n["fallbacks"] == 0

"""CPU pins of the oracle's chance-constrained verdict: a candidate is admissible
when the steady-state test passes and at most q of the N scenario rollouts
violate (the scenario approach with discarded samples, Sec. II-C).

* q = 0 is the robust verdict of Alg. 1 / Alg. 2, for the margin and the search;
* on linear plants every scenario's margin rows are affine in kappa, so each
  scenario admits exactly [0, kappa_k]; the number of violators at kappa is the
  number of kappa_k below it, and the largest admissible kappa is the
  (q + 1)-th smallest kappa_k (or the steady-state bound): bisection must
  return its dyadic floor;
* on nonlinear plants, the violator count and the order statistic against a
  brute-force count over single-scenario rollouts.
"""
import numpy as np
import pytest

from paper_2510_08288_amd import workloads as W


def _lq4_mats(p):
    c = p.coeffs
    return (c[0:16].reshape(4, 4), c[16:20], c[20:36].reshape(4, 4), c[36:44].reshape(4, 2),
            c[44:52].reshape(2, 4))


def _rk4_poly(A, h):
    Z = h * A
    I = np.eye(4)
    Z2 = Z @ Z
    Z3 = Z2 @ Z
    return I + Z + Z2 / 2 + Z3 / 6 + Z3 @ Z / 24, h * (I + Z / 2 + Z2 / 6 + Z3 / 24)


def _scenario_bounds(o, p, x0, r, v_prev, t):
    """kappa_k of every scenario (margin rows affine in kappa, ratio test over
    j = 0..H) and the steady-state bound, on a linear plant."""
    A, B, _, E, C = _lq4_mats(p)
    Phi, Psi = _rk4_poly(A, p.dt)
    F, g = p.F, p.g
    ks = []
    for k in range(p.N):
        xa, xb = x0.copy(), x0.copy()
        kk = np.inf
        for j in range(p.H + 1):
            a = g - F @ (C @ xa)
            b = g - F @ (C @ xb) - a
            assert np.all(a >= 0)
            for ai, bi in zip(a, b):
                if bi < 0:
                    kk = min(kk, -ai / bi)
            if j == p.H:
                break
            w = o.draw_w(t, k, j)
            xa = Phi @ xa + Psi @ (B * v_prev + E @ w)
            xb = Phi @ xb + Psi @ (B * r + E @ w)
        ks.append(kk)
    if not p.ss_check:
        return np.array(ks), np.inf
    H0 = -C @ np.linalg.solve(A, B)
    gt = g - p.eps * np.abs(g)
    a = gt - F @ (H0 * v_prev)
    b = gt - F @ (H0 * r) - a
    kss = np.inf
    for ai, bi in zip(a, b):
        if bi < 0:
            kss = min(kss, -ai / bi)
    return np.array(ks), kss


@pytest.mark.parametrize("kind", ["lq4", "fc9"])
def test_q0_is_the_robust_verdict(oracle_mod, kind):
    if kind == "lq4":
        p = W.lq4_problem(seed=24, N=24, H=300, dt=0.005, eps=0.01)
        x0, r, vp = np.zeros(4), 1.9, 0.0
    else:
        p = W.fc9_problem(N=24, H=200, dt=0.002)
        x0, r, vp = oracle_mod.Oracle(p).steady_margin(0.5)[1], 2.0, 0.5
    o = oracle_mod.Oracle(p)
    for kap in [0.0, 0.3, 0.75, 1.0]:
        v = o.candidate_v(kap, r, vp)
        M, per, _, _ = o.candidate(x0, v, 0)
        Mq, perq, nv = o.candidate_q(x0, v, 0, 0)
        assert Mq == M and np.array_equal(per, perq) and nv == int(np.sum(per < 0))
    a, b = o.bisect(x0, r, vp, 0, 12), o.bisect_q(x0, r, vp, 0, 12, 0)
    assert (a["kappa"], a["v"], a["passes"], a["status"]) == (b["kappa"], b["v"], b["passes"],
                                                              b["status"])


@pytest.mark.parametrize("seed,r", [(3, 2.6), (4, -2.0), (6, 2.5), (9, -1.2)])
def test_linear_plant_order_statistic(oracle_mod, seed, r):
    # steady-state test off, so the scenario rollouts alone decide
    p = W.lq4_problem(seed=seed, quad_scale=0.0, N=10, H=150, dt=0.01, w_half=0.3, ss_check=0)
    o = oracle_mod.Oracle(p)
    x0 = np.zeros(4)
    K = 12
    ks, kss = _scenario_bounds(o, p, x0, r, 0.0, 0)
    srt = np.sort(ks)
    assert kss == np.inf and srt[0] < srt[2] < srt[9] < 1.0
    for q in [0, 1, 2, 5, 9, 10, 12]:
        kq = srt[q] if q < p.N else np.inf
        kstar = min(kq, kss)
        res = o.bisect_q(x0, r, 0.0, 0, K, q)
        if kstar >= 1.0:
            assert res["kappa"] == 1.0 and res["passes"] == 1, q
            continue
        scaled = kstar * 2 ** K
        if abs(scaled - round(scaled)) < 1e-9:
            continue  # too close to a dyadic point to decide by arithmetic
        assert res["kappa"] == np.floor(scaled) / 2 ** K, (q, res["kappa"], kstar)
        # the violator count at the result and one dyadic above it
        _, _, nv = o.candidate_q(x0, o.candidate_v(res["kappa"], r, 0.0), 0, q)
        _, _, nv1 = o.candidate_q(x0, o.candidate_v(res["kappa"] + 2.0 ** -K, r, 0.0), 0, q)
        assert nv == int(np.sum(ks < res["kappa"])) and nv <= q
        assert nv1 == int(np.sum(ks < res["kappa"] + 2.0 ** -K))


@pytest.mark.parametrize("seed", [7, 12])
def test_count_and_order_statistic_brute_force(oracle_mod, seed):
    p = W.lq4_problem(seed=seed, N=8, H=100, dt=0.01, quad_scale=0.2)
    o = oracle_mod.Oracle(p)
    x0 = np.zeros(4)
    for kap in [0.25, 0.6, 1.0]:
        v = o.candidate_v(kap, 2.2, 0.0)
        per = np.array([o.rollout(x0, v, 0, k)[0] for k in range(p.N)])
        mss = o.steady_margin(v)[0]
        for q in range(p.N + 2):
            Mq, _, nv = o.candidate_q(x0, v, 0, q)
            assert nv == sum(1 for m in per if m < 0)
            mq = sorted(per)[q] if q < p.N else np.inf
            assert Mq == min(mq, mss)
            assert (Mq >= 0) == (nv <= q and mss >= 0)


def test_kappa_grows_with_q_and_saturates(oracle_mod):
    # a disturbance box wide enough that the scenario rollouts, not the
    # steady-state test, bind below q = N
    p = W.lq4_problem(seed=24, N=32, H=300, dt=0.005, eps=0.01, w_half=0.4)
    o = oracle_mod.Oracle(p)
    x0 = np.zeros(4)
    ks = [o.bisect_q(x0, 0.8, 0.3, 0, 10, q)["kappa"] for q in [0, 2, 8, 32]]
    assert ks == sorted(ks) and ks[0] < ks[1] < ks[2] < ks[3]
    # q >= N: only the steady-state test is left
    mss1 = o.steady_margin(0.8)[0]
    assert mss1 >= 0 and ks[-1] == 1.0

"""GPU parity on the 9-state plant: kappa of bisection and of the grid search
(Alg. 3 with refinement) against the FP64 oracle, both injection modes, streamed
vs inline draws, a short closed loop, and the full-size grid (N = 65536,
H = 1000) and adjoint (N = 16384, H = 1000) workloads checked on sampled
scenarios."""
import numpy as np
import pytest

from paper_2510_08288_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_GRAD = 1e-4


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2510_08288_amd import rg
    rg.load_library()
    return rg


def _start(o, v=0.5):
    return o.steady_margin(v)[1]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("inject", [W.INJECT_ODE, W.INJECT_POST])
def test_step_kappa_fc9(R, oracle_mod, precision, inject):
    # post-step injection adds w to every state once per step (not scaled by dt):
    # a 10x narrower box keeps kappa away from 0 there
    w_half = 0.02 if inject == W.INJECT_ODE else 0.002
    p = W.fc9_problem(N=300, H=250, dt=0.002, inject=inject, w_half=w_half)
    o = oracle_mod.Oracle(p, nthreads=8)
    x0 = _start(o)
    g = R.Governor(p, precision=precision)
    for t, r in [(0, 1.8), (1, 1.4), (2, 0.9)]:
        g.set_step(t)
        res = g.step(x0, r, 0.5)
        ref = o.bisect(x0, r, 0.5, t, 12)
        assert res["kappa"] == ref["kappa"], (t, r, res["kappa"], ref["kappa"])
        assert res["status"] == ref["status"] == 0
    g.close()


def test_grid_search_fc9(R, oracle_mod):
    p = W.fc9_problem(N=512, H=300, dt=0.002)
    o = oracle_mod.Oracle(p, nthreads=8)
    x0 = _start(o)
    for M, refine in [(64, 6), (17, 0)]:
        g = R.Governor(p, search=R.SEARCH_GRID, M=M, refine=refine)
        res = g.step(x0, 1.9, 0.5)
        ref = o.grid(x0, 1.9, 0.5, 0, M, refine)
        assert res["kappa"] == ref["kappa"] and res["status"] == ref["status"]
        assert res["bisect_passes"] == ref["passes"]
        g.close()


def test_stream_and_inline_draws_fc9(R):
    p = W.fc9_problem(N=200, H=150, dt=0.002)
    x0 = W.FC9_XBAR.copy()
    kap = np.array([0.25, 0.75])
    a = R.Governor(p, rng_mode=R.RNG_STREAM).margin(x0, 1.5, 0.5, kap, per_scenario=True)
    b = R.Governor(p, rng_mode=R.RNG_INLINE).margin(x0, 1.5, 0.5, kap, per_scenario=True)
    assert np.array_equal(a["per_scenario"], b["per_scenario"])
    assert np.array_equal(a["margins"], b["margins"])


def test_closed_loop_fc9(R, oracle_mod):
    p = W.fc9_problem(N=256, H=300, dt=0.002)
    o = oracle_mod.Oracle(p, nthreads=8)
    x0 = _start(o)
    r_seq = np.array([1.9, 1.9, 1.9, 1.2, 1.2, 2.0, 2.0, 0.8])
    g = R.Governor(p, K=10)
    out = g.closed_loop(x0, 0.5, r_seq, use_graph=True)
    v_prev = 0.5
    for s in range(len(r_seq)):
        ref = o.bisect(out["x"][s], r_seq[s], v_prev, s, 10)
        assert abs(out["kappa"][s] - ref["kappa"]) <= 2.0 ** -10, s
        xn = o.plant_step(out["x"][s], out["v"][s], s)
        np.testing.assert_allclose(out["x"][s + 1], xn, rtol=1e-13, atol=1e-14)
        v_prev = out["v"][s]
    g.close()


def _witness_checks(o, per, x0, kap, hi, r, vp, t):
    """The GPU's 8 worst scenarios at kap agree with the oracle one by one and
    are admissible; one scenario (or the steady state) refuses hi."""
    v0 = o.candidate_v(kap, r, vp)
    for k in np.argsort(per[0])[:8]:
        m = o.rollout(x0, v0, t, int(k))[0]
        assert abs(m - per[0][k]) <= TOL32 * max(1.0, abs(m)), (k, m, per[0][k])
        assert m >= 0.0 or kap == 0.0
    assert o.steady_margin(v0)[0] >= 0.0 or kap == 0.0
    if hi is not None:
        v1 = o.candidate_v(hi, r, vp)
        k1 = int(np.argmin(per[1]))
        assert min(o.rollout(x0, v1, t, k1)[0], o.steady_margin(v1)[0]) < 0.0


def _grid_bracket(kap, M, refine):
    """Upper end of the final bracket of Alg. 3 + `refine` halvings that ends at
    lower end kap: replays the halvings (grid points i/(M-1), midpoints
    (lo + hi) * 0.5) along the only verdict path that reaches kap."""
    if kap >= 1.0:
        return None
    i = max(i for i in range(M) if float(i) / float(M - 1) <= kap)
    lo, hi = float(i) / float(M - 1), float(i + 1) / float(M - 1)
    for _ in range(refine):
        mid = (lo + hi) * 0.5
        if kap >= mid:
            lo = mid
        else:
            hi = mid
    assert lo == kap
    return hi


def test_grid_full_size_sampled(R, oracle_mod):
    """64-point grid, 6 refinement halvings, FP32 with FP64 recheck, N = 65536, H = 1000."""
    p = W.fc9_problem(N=65536, H=1000, dt=0.002)
    o = oracle_mod.Oracle(p)
    x0 = _start(o)
    r, vp, M, refine = 2.0, 0.5, 64, 6
    g = R.Governor(p, search=R.SEARCH_GRID, M=M, refine=refine)
    res = g.step(x0, r, vp)
    assert res["status"] == 0
    kap = res["kappa"]
    hi = _grid_bracket(kap, M, refine)
    g.set_step(0)
    out = g.margin(x0, r, vp, [kap, hi if hi is not None else kap], per_scenario=True)
    _witness_checks(o, out["per_scenario"], x0, kap, hi, r, vp, 0)
    g.close()


def test_adjoint_full_size(R, oracle_mod):
    """Worst-margin gradient at N = 16384, H = 1000, checkpoints every 50 steps, and the
    Newton search against bisection on the same draws."""
    p = W.fc9_problem(N=16384, H=1000, dt=0.002)
    o = oracle_mod.Oracle(p, nthreads=8)
    x0 = _start(o)
    r, vp = 2.0, 0.5
    g = R.Governor(p, Kc=50)
    res = g.grad(x0, r, vp, 0.6)
    M, dk, dth, ka = o.candidate_grad(x0, 0.6, r, vp, 0)
    assert abs(res["M"] - M) <= TOL32 * max(1.0, abs(M))
    assert abs(res["dkappa"] - dk) <= TOL_GRAD * max(1.0, abs(dk))
    assert np.max(np.abs(res["dtheta"] - dth) / np.maximum(1.0, np.abs(dth))) <= TOL_GRAD
    g.set_step(0)
    kb = g.step(x0, r, vp)["kappa"]
    g.close()
    gn = R.Governor(p, search=R.SEARCH_NEWTON)
    kn = gn.step(x0, r, vp)["kappa"]
    gn.close()
    assert abs(kn - kb) <= 2.0 ** -12


def test_set_theta_refreshes_cached_steady_state(R, oracle_mod):
    O = oracle_mod
    # eps 0.45: the steady-state margin is the binding term.  The library keeps
    # the steady-state margins of recent set-points; new nominal coefficients
    # must replace them (both before and after the change the margins are the
    # FP64 oracle's for the coefficients in force).
    p = W.fc9_problem(N=128, H=300, dt=0.002).replace(eps=0.45)
    o = O.Oracle(p, nthreads=8)
    x0 = o.steady_margin(0.5)[1]
    co = p.coeffs.copy()
    co[90:110] *= 1.04
    o2 = O.Oracle(p.replace(coeffs=co), nthreads=8)
    g = R.Governor(p)
    kap = [1.0, 0.5]
    for ref_o, new in ((o, False), (o2, True), (o2, True)):
        if new:
            g.set_theta(co[90:110])
        g.set_step(0)
        m = g.margin(x0, 1.2, 0.5, kap)["margins"]
        for i, k in enumerate(kap):
            ref = ref_o.candidate(x0, ref_o.candidate_v(k, 1.2, 0.5), 0)[0]
            assert abs(m[i] - ref) <= 1e-9 * max(1.0, abs(ref)), (new, k, m[i], ref)
    g.close()


def test_fp64_tanh_within_3_ulp(R):
    # the project-written FP64 tanh of the 9-state plant's FP64 paths against an
    # extended-precision reference
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.prec = 120
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-1, 1, 4000) * 10.0 ** rng.uniform(-12, 1.4, 4000),
                        [0.0, -0.0, 1e-300, 0.3465735902799727, 0.35, -0.7, 19.99, 20.01, 50.0,
                         -50.0, np.inf, -np.inf, np.nan]])
    y = R.fp64_tanh(x)
    assert np.isnan(y[-1]) and y[-2] == -1.0 and y[-3] == 1.0 and y[-4] == -1.0
    assert y[4000] == 0.0 and y[4001] == 0.0 and np.signbit(y[4001])
    for xi, yi in zip(x[:-3], y[:-3]):
        ref = float(mpmath.tanh(mpmath.mpf(float(xi))))
        if ref == 0.0:
            assert yi == 0.0
            continue
        assert abs(yi - ref) <= 3 * np.spacing(abs(ref)), (xi, yi, ref)

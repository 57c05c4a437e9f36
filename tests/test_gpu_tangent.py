"""Forward-mode tangent fused into the FP32 rollout (rg_tangent,
RG_SEARCH_NEWTON_TAN) against the FP64 oracle's forward tangents of the
discrete RK4 map, the GPU adjoint, and bisection."""
import numpy as np
import pytest

from paper_2510_08288_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_GRAD = 1e-4   # FP32 tangent vs FP64 tangent, relative to max(1, |ref|)


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2510_08288_amd import rg
    rg.load_library()
    return rg


def _per_scenario(R, o, g, p, x0, r, vp, kap, t=0):
    g.set_step(t)
    res = g.tangent(x0, r, vp, kap)
    v = o.candidate_v(kap, r, vp)
    same_j = 0
    for k in range(p.N):
        m, dv, _, j, _ = o.rollout_tangent(x0, v, t, k)
        assert abs(res["m"][k] - m) <= TOL32 * max(1.0, abs(m)), (k, res["m"][k], m)
        if res["j"][k] == j:
            same_j += 1
            assert abs(res["dm_dv"][k] - dv) <= TOL_GRAD * max(1.0, abs(dv)), (k, res["dm_dv"][k], dv)
    # the FP32 and FP64 minimising steps agree except at near-ties
    assert same_j >= 0.9 * p.N, same_j
    return res


@pytest.mark.parametrize("lanes", [1, 4])
@pytest.mark.parametrize("inject", [0, 1])
@pytest.mark.parametrize("rng_mode", [0, 1])
def test_lq4_tangent_per_scenario(R, oracle_mod, lanes, inject, rng_mode):
    p = W.lq4_problem(seed=24, N=130, H=400, dt=0.005, eps=0.01, w_half=0.4, inject=inject)
    o = oracle_mod.Oracle(p, nthreads=8)
    g = R.Governor(p, lanes=lanes, rng_mode=rng_mode)
    assert g.options.lanes == lanes
    x0 = np.array([0.05, -0.1, 0.02, 0.1])
    for kap in [0.3, 1.0]:
        _per_scenario(R, o, g, p, x0, 1.6, 0.2, kap, t=2)
    g.close()


def test_fc9_tangent_per_scenario(R, oracle_mod):
    p = W.fc9_problem(N=96, H=300, dt=0.002, w_half=0.05)
    o = oracle_mod.Oracle(p, nthreads=8)
    x0 = o.steady_margin(0.5)[1]
    g = R.Governor(p)
    _per_scenario(R, o, g, p, x0, 2.0, 0.5, 0.4)
    g.close()


@pytest.mark.parametrize("kind", ["lq4", "fc9"])
def test_worst_margin_derivative_equals_adjoint(R, oracle_mod, kind):
    if kind == "lq4":
        p = W.lq4_problem(seed=24, N=256, H=500, dt=0.005, eps=0.01)
        x0, r, vp = np.zeros(4), 1.8, 0.0
        kaps = [0.25, 0.45, 0.9]
    else:
        p = W.fc9_problem(N=128, H=300, dt=0.002)
        x0 = oracle_mod.Oracle(p).steady_margin(0.5)[1]
        r, vp = 2.0, 0.5
        kaps = [0.3, 0.7]
    g = R.Governor(p, Kc=40)
    o = oracle_mod.Oracle(p, nthreads=8)
    for kap in kaps:
        tan = g.tangent(x0, r, vp, kap)
        adj = g.grad(x0, r, vp, kap)
        M, dk, _, _ = o.candidate_grad(x0, kap, r, vp, 0)
        assert abs(tan["M"] - adj["M"]) <= TOL32 * max(1.0, abs(adj["M"]))
        assert abs(tan["dkappa"] - adj["dkappa"]) <= TOL_GRAD * max(1.0, abs(adj["dkappa"]))
        assert abs(tan["dkappa"] - dk) <= TOL_GRAD * max(1.0, abs(dk)), (kap, tan["dkappa"], dk)
    g.close()


def test_tangent_margins_equal_plain_rollout(R):
    # the tangent lanes integrate the state with the operations of the plain
    # rollout: same FP32 margins
    p = W.lq4_problem(seed=24, N=200, H=300, dt=0.005, eps=0.01, w_half=0.4)
    for lanes in (1, 4):
        g = R.Governor(p, lanes=lanes)
        x0 = np.array([0.05, -0.1, 0.02, 0.1])
        tan = g.tangent(x0, 1.6, 0.2, 0.55)
        m = g.margin(x0, 1.6, 0.2, [0.55], per_scenario=True)["per_scenario"][0]
        err = np.abs(tan["m"] - m) / np.maximum(1.0, np.abs(m))
        assert float(np.max(err)) <= 1e-6, (lanes, float(np.max(err)))
        g.close()


@pytest.mark.parametrize("seed,r", [(24, 1.5), (24, -1.8), (10, 1.9), (19, -1.5), (7, 1.5)])
@pytest.mark.parametrize("lanes", [1, 4])
def test_tangent_newton_matches_bisection(R, oracle_mod, seed, r, lanes):
    p = W.lq4_problem(seed=seed, N=256, H=600, dt=0.005, eps=0.01)
    o = oracle_mod.Oracle(p, nthreads=8)
    g = R.Governor(p, search=R.SEARCH_NEWTON_TAN, lanes=lanes)
    res = g.step(np.zeros(4), r, 0.0)
    g.close()
    ref = o.bisect(np.zeros(4), r, 0.0, 0, 12)
    assert abs(res["kappa"] - ref["kappa"]) <= 2.0 ** -12
    assert res["rounds"] <= 14
    if 0 < res["kappa"] < 1:
        M = o.candidate(np.zeros(4), o.candidate_v(res["kappa"], r, 0.0), 0)[0]
        assert M >= -1e-5   # admissible up to the FP32 margin tolerance


def test_tangent_newton_fc9(R, oracle_mod):
    p = W.fc9_problem(N=128, H=400, dt=0.002)
    o = oracle_mod.Oracle(p, nthreads=8)
    x0 = o.steady_margin(0.5)[1]
    g = R.Governor(p, search=R.SEARCH_NEWTON_TAN)
    res = g.step(x0, 2.0, 0.5)
    g.close()
    ref = o.bisect(x0, 2.0, 0.5, 0, 12)
    assert abs(res["kappa"] - ref["kappa"]) <= 2.0 ** -12


def test_tangent_newton_closed_loop(R, oracle_mod):
    p = W.lq4_problem(seed=24, N=256, H=400, dt=0.005, eps=0.01)
    r_seq = W.reference_sequence(7, 16, switch_every=4)
    a = R.Governor(p, search=R.SEARCH_NEWTON_TAN).closed_loop(np.zeros(4), 0.0, r_seq,
                                                              use_graph=True)
    b = R.Governor(p, search=R.SEARCH_NEWTON_TAN).closed_loop(np.zeros(4), 0.0, r_seq,
                                                              use_graph=False)
    assert np.array_equal(a["kappa"], b["kappa"]) and np.array_equal(a["x"], b["x"])
    o = oracle_mod.Oracle(p, nthreads=8)
    v_prev = 0.0
    for s in range(len(r_seq)):
        ref = o.bisect(a["x"][s], r_seq[s], v_prev, s, 12)
        assert abs(a["kappa"][s] - ref["kappa"]) <= 2.0 ** -12, s
        v_prev = a["v"][s]

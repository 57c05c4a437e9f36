"""GPU checks of the 9-state rollouts by groups of 16 lanes (one lane per
state component), in the FP64 recheck of near-band scenarios and in FP32
rounds with few scenarios:

* FP64 recheck: its margins equal, bit for bit, those of the one-lane FP64
  rollouts (F64 precision) of the same scenarios, for both injection modes and
  both draw modes, with a band wide enough that every scenario is rechecked;
  on the grid search of the paper-shaped timing workload (M = 32, H = 1024)
  at an N whose returned row has a near-band scenario, the FP32 + recheck
  search returns the kappa of the all-FP64 search;
* FP32 rollouts (lanes = 16): per-scenario margins and minimising steps equal
  the one-lane kernel's bit for bit (ragged N, both injections, both draw
  modes); grid and bisection kappa equal the oracle's; the adjoint built on
  the groups' checkpoints equals the one built on one-lane checkpoints; the
  automatic layout takes groups only for rounds of few scenarios."""
import numpy as np
import pytest

from paper_2510_08288_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2510_08288_amd import rg
    rg.load_library()
    return rg


@pytest.mark.parametrize("inject", [W.INJECT_ODE, W.INJECT_POST])
@pytest.mark.parametrize("rng_mode", [0, 1])
def test_group_recheck_equals_one_lane_fp64(R, inject, rng_mode):
    w_half = 0.02 if inject == W.INJECT_ODE else 0.002
    p = W.fc9_problem(N=61, H=400, dt=0.002, inject=inject, w_half=w_half)
    # a start away from equilibrium, so that the rollouts (not the
    # steady-state term) set the margins
    x0 = W.FC9_XBAR + np.array([0.05, -0.04, 0.03, 0.0, -0.02, 0.01, 0.08, 0.0, -0.05])
    kap = np.array([0.0, 0.3, 0.6, 1.0])
    print(f"[recheck] inject={inject} rng_mode={rng_mode} N=61 H=400 M=4", flush=True)
    wide = R.Governor(p, band=1e30, rng_mode=rng_mode)
    a = wide.margin(x0, 1.9, 0.5, kap, per_scenario=True)
    wide.close()
    f64 = R.Governor(p, precision=R.PREC_F64, rng_mode=rng_mode)
    b = f64.margin(x0, 1.9, 0.5, kap, per_scenario=True)
    f64.close()
    assert np.array_equal(a["margins"], b["margins"]), (a["margins"], b["margins"])
    # the rollouts decide every margin here (the steady-state term is above)
    per = np.asarray(b["per_scenario"], dtype=np.float64).reshape(len(kap), -1)
    assert np.allclose(per.min(axis=1), b["margins"], rtol=1e-6, atol=1e-6)


def test_grid_recheck_keeps_fp64_kappa(R):
    p = W.fc9_problem(N=1312, H=1024, dt=0.01)
    print("[recheck] grid M=32 N=1312 H=1024", flush=True)
    g = R.Governor(p, search=R.SEARCH_GRID, M=32, refine=0)
    x0 = g.equilibrium(0.5)
    res = g.step(x0, 2.0, 0.5)
    g.close()
    g64 = R.Governor(p, precision=R.PREC_F64, search=R.SEARCH_GRID, M=32, refine=0)
    ref = g64.step(x0, 2.0, 0.5)
    g64.close()
    assert res["rechecks"] >= 1
    assert res["kappa"] == ref["kappa"] and res["status"] == ref["status"] == 0


@pytest.mark.parametrize("inject", [W.INJECT_ODE, W.INJECT_POST])
@pytest.mark.parametrize("rng_mode", [0, 1])
def test_fp32_groups_equal_one_lane(R, inject, rng_mode):
    w_half = 0.02 if inject == W.INJECT_ODE else 0.002
    p = W.fc9_problem(N=61, H=300, dt=0.002, inject=inject, w_half=w_half)
    x0 = W.FC9_XBAR + np.array([0.05, -0.04, 0.03, 0.0, -0.02, 0.01, 0.08, 0.0, -0.05])
    kap = np.array([0.0, 0.2, 0.5, 0.8, 1.0])
    print(f"[groups] fp32 inject={inject} rng_mode={rng_mode} N=61 H=300 M=5", flush=True)
    out = {}
    for lanes in (1, 16):
        g = R.Governor(p, lanes=lanes, rng_mode=rng_mode)
        assert g.options.lanes == lanes
        out[lanes] = g.margin(x0, 1.9, 0.5, kap, per_scenario=True)
        g.close()
    assert np.array_equal(out[1]["per_scenario"], out[16]["per_scenario"])
    assert np.array_equal(out[1]["per_scenario_j"], out[16]["per_scenario_j"])
    assert np.array_equal(out[1]["margins"], out[16]["margins"])


def test_fp32_groups_search_kappa(R, oracle_mod):
    p = W.fc9_problem(N=40, H=400, dt=0.002)
    o = oracle_mod.Oracle(p, nthreads=8)
    x0 = o.steady_margin(0.5)[1]
    print("[groups] grid and bisection N=40 H=400", flush=True)
    g = R.Governor(p, lanes=16, search=R.SEARCH_GRID, M=32, refine=3)
    res = g.step(x0, 1.9, 0.5)
    g.close()
    ref = o.grid(x0, 1.9, 0.5, 0, 32, 3)
    assert res["kappa"] == ref["kappa"] and res["status"] == ref["status"]
    g = R.Governor(p, lanes=16)
    for t, r in [(0, 1.8), (1, 1.4), (2, 0.9)]:
        g.set_step(t)
        res = g.step(x0, r, 0.5)
        ref = o.bisect(x0, r, 0.5, t, 12)
        assert res["kappa"] == ref["kappa"] and res["status"] == ref["status"] == 0
    g.close()


def test_fp32_groups_adjoint_checkpoints(R):
    p = W.fc9_problem(N=48, H=300, dt=0.002)
    x0 = W.FC9_XBAR + np.array([0.05, -0.04, 0.03, 0.0, -0.02, 0.01, 0.08, 0.0, -0.05])
    print("[groups] adjoint on group checkpoints N=48 H=300", flush=True)
    out = {}
    for lanes in (1, 16):
        g = R.Governor(p, lanes=lanes, search=R.SEARCH_NEWTON)
        out[lanes] = (g.grad(x0, 1.9, 0.5, 0.4), g.step(x0, 1.9, 0.5)["kappa"])
        g.close()
    a, b = out[1][0], out[16][0]
    assert a["M"] == b["M"] and a["dkappa"] == b["dkappa"]
    assert np.array_equal(a["dtheta"], b["dtheta"])
    assert out[1][1] == out[16][1]


def test_auto_lanes_choose_groups_for_small_rounds(R):
    small = R.Governor(W.fc9_problem(N=64, H=100), search=R.SEARCH_GRID, M=32, refine=0)
    large = R.Governor(W.fc9_problem(N=4096, H=100), search=R.SEARCH_GRID, M=32, refine=0)
    tan = R.Governor(W.fc9_problem(N=64, H=100), search=R.SEARCH_NEWTON_TAN)
    assert (small.options.lanes, large.options.lanes, tan.options.lanes) == (16, 1, 1)
    for g in (small, large, tan):
        g.close()


@pytest.mark.parametrize("N,H", [(1, 1), (1, 200), (17, 3), (257, 5), (33, 150)])
def test_fp32_groups_edge_sizes(R, oracle_mod, N, H):
    # one group, ragged workgroups (16 scenarios per 256 lanes), short horizons
    p = W.fc9_problem(N=N, H=H, dt=0.002)
    x0 = W.FC9_XBAR + np.array([0.05, -0.04, 0.03, 0.0, -0.02, 0.01, 0.08, 0.0, -0.05])
    kap = np.array([0.1, 0.7])
    print(f"[groups] edge N={N} H={H}", flush=True)
    out = {}
    for lanes in (1, 16):
        g = R.Governor(p, lanes=lanes)
        out[lanes] = g.margin(x0, 1.9, 0.5, kap, per_scenario=True)
        g.close()
    assert np.array_equal(out[1]["per_scenario"], out[16]["per_scenario"])
    assert np.array_equal(out[1]["margins"], out[16]["margins"])
    o = oracle_mod.Oracle(p, nthreads=4)
    xs = o.steady_margin(0.5)[1]
    g = R.Governor(p, lanes=16)
    res = g.step(xs, 1.9, 0.5)
    g.close()
    ref = o.bisect(xs, 1.9, 0.5, 0, 12)
    assert res["kappa"] == ref["kappa"] and res["status"] == ref["status"]


def test_flat_recheck_wide_band_both_layouts(R, oracle_mod):
    # batched serving: a band wider than every margin makes the FP64 recheck
    # give every verdict; with one candidate per round the instances with at
    # most 8 entries run the group form of the flat recheck, the N = 40
    # instance the one-lane form.  kappa must be the FP64 oracle's.
    Ns = [2, 3, 4, 40]
    probs = [W.fc9_problem(N=N, H=300, dt=0.002, scen_seed=300 + i, instance=i)
             for i, N in enumerate(Ns)]
    x0 = oracle_mod.Oracle(probs[0]).steady_margin(0.5)[1]
    xs, rs, vps = [x0] * len(Ns), [1.9, 1.7, 1.5, 1.9], [0.5] * len(Ns)
    print("[groups] flat recheck, wide band, N =", Ns, flush=True)
    b = R.Batch(probs, band=50.0, depth=1)
    out = b.step(xs, rs, vps, use_graph=False)
    b.close()
    for i, p in enumerate(probs):
        ref = oracle_mod.Oracle(p, nthreads=8).bisect(xs[i], rs[i], vps[i], 0, 12)
        assert out["kappa"][i] == ref["kappa"], (i, out["kappa"][i], ref["kappa"])
        assert out["status"][i] == ref["status"]

"""GPU checks of the FP64 recheck of the 9-state plant, which re-simulates a few
near-band scenarios with one lane per state component (groups of 16 lanes):

* its margins equal, bit for bit, those of the one-lane FP64 rollouts (F64
  precision) of the same scenarios, for both injection modes and both draw
  modes, with a band wide enough that every scenario is rechecked;
* on the grid search of the paper-shaped timing workload (M = 32, H = 1024)
  at an N whose returned row has a near-band scenario, the FP32 + recheck
  search returns the kappa of the all-FP64 search."""
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

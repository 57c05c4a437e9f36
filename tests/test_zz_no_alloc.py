"""rg_step_noalloc (the RG step that allocates nothing: static device scratch,
draws regenerated in the kernels) against rg_step on its own handle, through
the C ABI: two calls in a row on the same GPU, the second with a smaller
problem, so the second call runs on whatever the first left in the shared
scratch."""
import numpy as np
import pytest

from paper_2510_08288_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2510_08288_amd import rg
    rg.load_library()
    return rg


def _compare(R, p, x, r, vp, t, **kw):
    a = R.Governor(p, torch_workspace=False, **kw)   # never given a workspace
    a.set_step(t)
    got = a.step_noalloc(x, r, vp)
    assert a.get_step() == t + 1
    a.close()
    b = R.Governor(p, **kw)
    b.set_step(t)
    ref = b.step(x, r, vp)
    b.close()
    assert got["kappa"] == ref["kappa"], (got["kappa"], ref["kappa"])
    assert got["v"] == ref["v"] and got["status"] == ref["status"]
    assert got["bisect_passes"] == ref["bisect_passes"] and got["t"] == t
    if np.isfinite(ref["worst"]):
        assert abs(got["worst"] - ref["worst"]) <= TOL32 * max(1.0, abs(ref["worst"]))
    else:
        assert got["worst"] == ref["worst"]
    return got


def test_two_calls_second_smaller(R):
    # first: the 4-state bench workload (N = 4096, H = 2000) at a state where
    # the search runs (kappa strictly between 0 and 1)
    wl = W.workload_lq4_closed_loop(T=40)
    x = np.array([0.12, -0.05, 0.3, -0.2])
    big = _compare(R, wl["problem"], x, 1.9, 0.4, 26, band=wl["band"], K=wl["K"])
    assert 0.0 < big["kappa"] < 1.0 and big["bisect_passes"] == 13
    # second, smaller: N = 300, H = 400, a wide disturbance box
    p = W.lq4_problem(seed=24, N=300, H=400, dt=0.005, eps=0.01, w_half=0.4)
    small = _compare(R, p, np.zeros(4), 0.8, 0.3, 3)
    assert 0.0 < small["kappa"] < 1.0


@pytest.mark.parametrize("kind", ["fc9", "grid", "fp64", "infeasible"])
def test_other_forms(R, oracle_mod, kind):
    if kind == "fc9":
        p = W.fc9_problem(N=256, H=300, dt=0.002, w_half=0.05)
        x = oracle_mod.Oracle(p).steady_margin(0.5)[1]
        _compare(R, p, x, 2.0, 0.5, 1)
    elif kind == "grid":
        p = W.lq4_problem(seed=24, N=200, H=300, dt=0.005, eps=0.01, w_half=0.4)
        _compare(R, p, np.zeros(4), 0.8, 0.3, 0, search=R.SEARCH_GRID, M=16, refine=4)
    elif kind == "fp64":
        p = W.lq4_problem(seed=24, N=64, H=500, dt=0.01, eps=0.05)
        _compare(R, p, np.zeros(4), 1.5, 0.0, 0, precision=R.PREC_F64)
    else:
        p = W.lq4_problem(seed=24, N=96, H=100, dt=0.005, eps=0.01, w_half=0.4)
        C = np.asarray(p.coeffs[44:52]).reshape(2, 4)
        got = _compare(R, p, 3.0 * C[0] / float(C[0] @ C[0]), 0.5, 0.1, 0)
        assert got["status"] == R.RG_S_INFEASIBLE and got["v"] == 0.1


def test_refusals(R):
    # recheck list beyond the static scratch: 64 grid points x 65536 scenarios
    p = W.fc9_problem(N=65536, H=10)
    g = R.Governor(p, search=R.SEARCH_GRID, M=64, torch_workspace=False)
    with pytest.raises(R.RGError) as e:
        g.step_noalloc(np.asarray(W.FC9_XBAR), 1.0, 0.5)
    assert e.value.code == R.RG_E_NOTSUP and "scratch" in str(e.value)
    g.close()
    g = R.Governor(W.lq4_problem(N=64, H=50), search=R.SEARCH_NEWTON, torch_workspace=False)
    with pytest.raises(R.RGError) as e:
        g.step_noalloc(np.zeros(4), 1.0, 0.0)
    assert e.value.code == R.RG_E_NOTSUP
    g.close()

"""Full-size parity of the named workloads against the FP64 oracle.

* The 4-state bench workload (N = 4096, H = 2000, 200 closed-loop RG updates):
  kappa of every update equals the FP64 oracle's own closed loop, stored in
  tests/golden/lq4_closed_loop_n4096_h2000.txt by a script that calls only the
  oracle; states and set-points follow it.
* All 4096 per-scenario FP32 margins of one full-horizon candidate against the
  oracle's rollouts, element by element (1e-5 relative).
* The 9-state grid workload (N = 65536, H = 1000, Alg. 3 with 64 points and 6
  refinements): every scenario admits the result (oracle over all 65536
  rollouts), and the end of the final bracket is refused by some scenario or by
  the steady-state test.
"""
import os

import numpy as np
import pytest

from paper_2510_08288_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
THREADS = min(16, os.cpu_count() or 1)
FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "lq4_closed_loop_n4096_h2000.txt")


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2510_08288_amd import rg
    rg.load_library()
    return rg


def _fixture():
    rows = np.array([[float(c) for c in ln.split()] for ln in open(FIXTURE)
                     if ln.strip() and not ln.startswith("#")])
    return dict(t=rows[:, 0].astype(int), r=rows[:, 1], v_prev=rows[:, 2], x=rows[:, 3:7],
                kappa=rows[:, 7], v=rows[:, 8], passes=rows[:, 9].astype(int),
                status=rows[:, 10].astype(int))


@pytest.mark.parametrize("use_graph", [True, False])
def test_bench_closed_loop_equals_oracle_fixture(R, use_graph):
    wl = W.workload_lq4_closed_loop(T=200)
    ref = _fixture()
    assert len(ref["kappa"]) == 200
    np.testing.assert_array_equal(ref["r"], wl["r_seq"])
    g = R.Governor(wl["problem"], band=wl["band"], K=wl["K"])
    out = g.closed_loop(wl["x0"], wl["v_prev"], wl["r_seq"], use_graph=use_graph)
    g.close()
    # the search does not stop at a boundary-holding regime only: the loop has
    # updates at kappa = 1, at kappa = 0 and strictly between
    assert np.any(ref["kappa"] == 1.0) and np.any(ref["kappa"] == 0.0)
    assert np.any((ref["kappa"] > 0.0) & (ref["kappa"] < 1.0))
    bad = np.nonzero(out["kappa"] != ref["kappa"])[0]
    assert bad.size == 0, [(int(s), out["kappa"][s], ref["kappa"][s]) for s in bad[:5]]
    np.testing.assert_array_equal(out["v"], ref["v"])
    # the true plant is stepped in FP64 by both sides (different operation order)
    np.testing.assert_allclose(out["x"][:200], ref["x"], rtol=1e-11, atol=1e-13)
    assert np.array_equal(out["status"] != 0, ref["status"] != 0)
    assert np.array_equal(out["bisect_passes"], ref["passes"])


def test_full_size_margins_every_scenario(R, oracle_mod):
    wl = W.workload_lq4_closed_loop(T=2)
    p = wl["problem"]
    o = oracle_mod.Oracle(p, nthreads=THREADS)
    x0 = np.array([0.12, -0.05, 0.3, -0.2])
    r, vp = 1.9, 0.4
    g = R.Governor(p, band=wl["band"], K=wl["K"])
    kappas = [0.0, 0.37109375, 1.0]
    out = g.margin(x0, r, vp, kappas, per_scenario=True)
    g.close()
    for i, kap in enumerate(kappas):
        M, per, _, mss = o.candidate(x0, o.candidate_v(kap, r, vp), 0)
        gpu = out["per_scenario"][i].astype(np.float64)
        err = np.abs(gpu - per) / np.maximum(1.0, np.abs(per))
        assert float(np.max(err)) <= TOL32, (kap, float(np.max(err)), int(np.argmax(err)))
        assert abs(out["margins"][i] - M) <= TOL32 * max(1.0, abs(M))


def _grid_upper(kap, M, refine):
    """Upper end of the final bracket of Alg. 3 + `refine` halvings ending at kap."""
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


def test_fc9_grid_full_size_every_scenario(R, oracle_mod):
    wl = W.workload_fc9_grid()
    p = wl["problem"]
    o = oracle_mod.Oracle(p, nthreads=THREADS)
    g = R.Governor(p, search=R.SEARCH_GRID, M=wl["M"], refine=wl["refine"], band=wl["band"])
    x0 = g.equilibrium(wl["v_prev"])
    np.testing.assert_allclose(x0, o.steady_margin(wl["v_prev"])[1], rtol=1e-11, atol=1e-12)
    r, vp = wl["r"], wl["v_prev"]
    res = g.step(x0, r, vp)
    g.close()
    assert res["status"] == 0
    kap = res["kappa"]
    hi = _grid_upper(kap, wl["M"], wl["refine"])
    M_lo, per_lo, _, mss_lo = o.candidate(x0, o.candidate_v(kap, r, vp), 0)
    assert np.all(per_lo >= 0.0) and mss_lo >= 0.0, (float(np.min(per_lo)), mss_lo)
    if hi is not None:
        M_hi, per_hi, _, mss_hi = o.candidate(x0, o.candidate_v(hi, r, vp), 0)
        assert M_hi < 0.0
        # the refusal is not an artefact of the FP32 band: some scenario or the
        # steady state is below zero in FP64
        assert np.any(per_hi < 0.0) or mss_hi < 0.0

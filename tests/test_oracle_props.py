"""Property tests of the FP64 CPU reference over random tiny problems.

The fixed-seed pins elsewhere check the reference on chosen cases; these draw
plants, scenario sets, horizons, references and search depths at random
(hypothesis, derandomized so that every run checks the same examples) and
check invariants that Alg. 1 and the scenario construction fix whatever the
plant:

* the bisection bracket: kappa is a multiple of 2^-K, an admitted result is
  admissible, and kappa + 2^-K is refused whenever kappa < 1;
* more scenarios or a longer horizon never admit more (the draws of a smaller
  problem are a prefix of the larger one's);
* on linear plants from an admissible state, Alg. 2 (per-scenario bisection,
  then the minimum) returns the same kappa as the joint bisection of Alg. 1;
* kappa = 1 returns v = r exactly, and v = v_prev + kappa (r - v_prev);
* the chance-constrained verdict admits no less as q grows, and q = 0 is the
  robust verdict.
"""
import numpy as np
from hypothesis import assume, given, settings, strategies as st

from paper_2510_08288_amd import workloads as W

SETTINGS = settings(max_examples=25, deadline=None, derandomize=True)

plant_seed = st.integers(min_value=0, max_value=10_000)
scen_seed = st.integers(min_value=0, max_value=2**31 - 1)
ref = st.floats(min_value=-2.5, max_value=2.5, allow_nan=False)
vprev = st.floats(min_value=-0.3, max_value=0.3, allow_nan=False)
depth = st.integers(min_value=1, max_value=8)


def _problem(seed, sseed, N, H, w_half=0.05, quad_scale=0.05):
    return W.lq4_problem(seed=seed, N=N, H=H, dt=0.01, w_half=w_half, eps=0.01,
                         quad_scale=quad_scale, scen_seed=sseed)


@SETTINGS
@given(seed=plant_seed, sseed=scen_seed, N=st.integers(1, 12), H=st.integers(1, 60), r=ref,
       vp=vprev, K=depth)
def test_bisection_bracket_invariant(oracle_mod, seed, sseed, N, H, r, vp, K):
    o = oracle_mod.Oracle(_problem(seed, sseed, N, H))
    x0 = np.zeros(4)
    res = o.bisect(x0, r, vp, 0, K)
    kap = res["kappa"]
    assert 0.0 <= kap <= 1.0
    assert kap * 2**K == np.floor(kap * 2**K)  # a dyadic of depth K
    assert res["v"] == o.candidate_v(kap, r, vp)
    if res["status"] == 0:
        assert o.candidate(x0, res["v"], 0)[0] >= 0.0
    if kap < 1.0:
        above = o.candidate_v(kap + 2.0**-K, r, vp)
        assert o.candidate(x0, above, 0)[0] < 0.0
    if kap == 1.0:
        assert res["v"] == r


@SETTINGS
@given(seed=plant_seed, sseed=scen_seed, N1=st.integers(1, 6), dN=st.integers(1, 10),
       H1=st.integers(1, 40), dH=st.integers(1, 40), r=ref, K=depth)
def test_more_scenarios_or_steps_never_admit_more(oracle_mod, seed, sseed, N1, dN, H1, dH, r, K):
    x0 = np.zeros(4)
    k = {}
    for key, (N, H) in {"small": (N1, H1), "moreN": (N1 + dN, H1),
                        "moreH": (N1, H1 + dH)}.items():
        k[key] = oracle_mod.Oracle(_problem(seed, sseed, N, H)).bisect(x0, r, 0.0, 0, K)["kappa"]
    assert k["moreN"] <= k["small"]
    assert k["moreH"] <= k["small"]


@SETTINGS
@given(seed=plant_seed, sseed=scen_seed, N=st.integers(1, 8), H=st.integers(5, 60), r=ref,
       K=depth)
def test_alg2_equals_bisection_on_linear_plants(oracle_mod, seed, sseed, N, H, r, K):
    # linear plant (no quadratic term): every scenario margin is concave in v,
    # so from an admissible start each admissible set of kappa is an interval
    # [0, kappa*] and the per-scenario bisections meet the joint one
    o = oracle_mod.Oracle(_problem(seed, sseed, N, H, quad_scale=0.0))
    x0 = np.zeros(4)
    assume(o.candidate(x0, 0.0, 0)[0] >= 0.0)  # kappa = 0 admissible: an interval [0, kappa*]
    a = o.bisect(x0, r, 0.0, 0, K)
    b = o.alg2(x0, r, 0.0, 0, K)
    assert a["kappa"] == b["kappa"]


@SETTINGS
@given(seed=plant_seed, sseed=scen_seed, N=st.integers(1, 12), H=st.integers(1, 50), r=ref,
       K=depth, q1=st.integers(0, 6), dq=st.integers(0, 8))
def test_chance_verdict_monotone_in_q(oracle_mod, seed, sseed, N, H, r, K, q1, dq):
    # admitting up to q violating scenarios admits at least what q' < q admits,
    # and q = 0 is the robust verdict
    o = oracle_mod.Oracle(_problem(seed, sseed, N, H, w_half=0.3))
    x0 = np.zeros(4)
    a = o.bisect_q(x0, r, 0.0, 0, K, q1)
    b = o.bisect_q(x0, r, 0.0, 0, K, q1 + dq)
    assert a["kappa"] <= b["kappa"]
    if q1 == 0:
        assert a["kappa"] == o.bisect(x0, r, 0.0, 0, K)["kappa"]

"""CPU pins of the oracle's 9-state plant (FC9): right-hand side, outputs and
the steady state, each checked against something other than the oracle's own
formula.

The paper's fuel-cell model is only cited (Sec. IV-A), so FC9 is this project's
stand-in; its definition is restated in the oracle header and in include/rg.h.
The pins below come from that definition by hand, not from a second
transcription of the right-hand side:

* at x = xbar the tanh coupling vanishes, so every derivative is a short
  expression in the nominal coefficients (values worked out by hand);
* with W = 0 and a_1..a_6 = 0 the equilibrium has a closed form: every orifice
  carries the compressor flow q = c_q0 w1, the pressures follow by summing
  (q / k_l)^2 from p_amb upwards, w2 and w3 are explicit, and w1 is the single
  real root of a cubic (numpy.roots);
* the flows of the volume chain telescope, a single entry of W shows up as one
  tanh term in one row, and a closed check valve (p_l <= p_{l+1}) makes the
  downstream derivative independent of p_l.
"""
import numpy as np
import pytest

from paper_2510_08288_amd import workloads as W

def _plant(**kw):
    return W.fc9_problem(N=1, H=10, w_half=0.0, theta_rel=0.0, **kw)


def _special(k=(3.0, 2.5, 2.8, 3.2, 2.6, 3.0)):
    """W = 0, a_1..a_6 = 0 (through the nominal coefficients), orifice gains k;
    the other coefficients get pairwise distinct values so that a swapped index
    changes the result."""
    p = _plant()
    co = p.coeffs.copy()
    co[:81] = 0.0
    co[90:96] = 0.0
    co[96:99] = (2.2, 3.1, 11.0)      # a_7..a_9
    co[99:105] = k
    co[105:108] = (1.3, 0.6, 5.0)     # b_1..b_3
    co[108:110] = (0.45, 0.8)         # mu_1, mu_2
    co[110:115] = (0.65, 1.05, 0.06, 0.3, 1.55)  # c_q0, p_amb, d0, d1, p1ref
    return p.replace(coeffs=co)


def test_fc9_rhs_at_xbar_hand_values(oracle_mod):
    # z = 0: tanh(z) = 0 removes W and the -a z terms.  Pressures 1.6 .. 1.1 and
    # p_amb = 1 give dp = 0.1 at every orifice (k = 1), so q_l = sqrt(0.1) for
    # l = 1..6 and q_0 = c_q0 w1 = 0.7; the bilinear rows use b = (1.5, 0.5, 6),
    # mu = (0.5, 0.5), w1 = w3 = 1 and p1 = p1ref.
    p = _plant()
    o = oracle_mod.Oracle(p)
    xbar = W.FC9_XBAR
    s01 = np.sqrt(0.1)
    for v in [0.0, 0.7, 1.9]:
        xd = o.rhs(xbar, v, np.zeros(9))
        expect = np.array([0.7 - s01, 0, 0, 0, 0, 0, 1.5 * v, 0.5 * v, 6.0 * v])
        np.testing.assert_allclose(xd, expect, rtol=0, atol=2e-15)
    # an additive disturbance enters each row once, with unit gain
    w = np.linspace(-0.02, 0.02, 9)
    np.testing.assert_allclose(o.rhs(xbar, 0.7, w) - o.rhs(xbar, 0.7, np.zeros(9)), w,
                               rtol=0, atol=2e-15)


def test_fc9_output_hand_values(oracle_mod):
    # y = (c_q0 w1 / (d0 + d1 w3), p1, w1) with c_q0 = 0.7, d0 = 0.05, d1 = 0.25;
    # every state gets a distinct value so a wrong index shows.
    p = _plant()
    o = oracle_mod.Oracle(p)
    x = np.array([2.05, 1.91, 1.77, 1.63, 1.49, 1.35, 1.2, 1.11, 1.8])
    y = o.output(x, 0.4)
    assert y[0] == pytest.approx(0.84 / 0.5, rel=1e-15)      # 0.7 * 1.2 / (0.05 + 0.45)
    assert y[1] == 2.05 and y[2] == 1.2
    x2 = x.copy()
    x2[7] = 5.0   # w2 enters no output
    np.testing.assert_array_equal(o.output(x2, 0.4), y)
    x2[8] = 0.2   # w3 only in the ratio's denominator
    assert o.output(x2, 0.4)[0] == pytest.approx(0.84 / 0.1, rel=1e-15)


@pytest.mark.parametrize("v", [0.3, 0.8, 1.4])
def test_fc9_equilibrium_closed_form(oracle_mod, v):
    p = _special()
    o = oracle_mod.Oracle(p)
    c_q0, p_amb, d0, d1, p1ref = p.coeffs[110:115]
    th = p.coeffs[90:110]
    a, k, b, mu = th[:9], th[9:15], th[15:18], th[18:20]
    xbar = p.coeffs[81:90]
    S = np.sum(1.0 / k ** 2)
    # w1 row: -a7 (w1 - xbar7) + b1 v - mu1 w1 (p1 - p1ref) = 0 with
    # p1 = p_amb + (c_q0 w1)^2 S; the cubic is strictly decreasing (one real root)
    cubic = [-mu[0] * c_q0 ** 2 * S, 0.0, -(a[6] + mu[0] * (p_amb - p1ref)),
             a[6] * xbar[6] + b[0] * v]
    roots = np.roots(cubic)
    real = [r.real for r in roots if abs(r.imag) < 1e-9 * max(1.0, abs(r))]
    assert len(real) == 1
    w1 = real[0]
    q = c_q0 * w1
    pr = np.empty(7)
    pr[6] = p_amb
    for l in range(5, -1, -1):
        pr[l] = pr[l + 1] + (q / k[l]) ** 2
    w2 = xbar[7] + b[1] * v * w1 / a[7]
    w3 = (a[8] * xbar[8] + b[2] * v + mu[1] * v) / (a[8] + mu[1] * v)
    x_cf = np.concatenate([pr[:6], [w1, w2, w3]])
    m, xs, it = o.steady_margin(v)
    np.testing.assert_allclose(xs, x_cf, rtol=1e-12, atol=1e-12)
    assert it <= 8   # Newton with the analytic Jacobian converges quadratically
    y1 = c_q0 * w1 / (d0 + d1 * w3)
    y = np.array([y1, pr[0], w1])
    rows = p.g - p.eps * np.abs(p.g) - p.F @ y
    assert m == pytest.approx(np.min(rows), abs=1e-12)


def test_fc9_flows_telescope(oracle_mod):
    # With W = 0 and a_1..a_6 = 0 the six pressure rows are q_{l-1} - q_l, so
    # their sum is q_0 - q_6 = c_q0 w1 - k_6 sqrt(max(p6 - p_amb, 0)) whatever
    # the intermediate pressures.
    p = _special()
    o = oracle_mod.Oracle(p)
    c_q0, p_amb = p.coeffs[110:112]
    k6 = p.coeffs[104]
    rng = np.random.default_rng(4)
    for _ in range(20):
        x = np.concatenate([np.sort(rng.uniform(1.0, 2.5, 6))[::-1], rng.uniform(0.5, 2.0, 3)])
        x[:6] += rng.uniform(-0.2, 0.2, 6) * (rng.uniform(size=6) < 0.3)  # some valves closed
        xd = o.rhs(x, rng.uniform(0, 2), np.zeros(9))
        q6 = k6 * np.sqrt(max(x[5] - p_amb, 0.0))
        assert np.sum(xd[:6]) == pytest.approx(c_q0 * x[6] - q6, abs=1e-13)


def test_fc9_coupling_single_entry(oracle_mod):
    # W = c e_i e_j^T adds c tanh(x_j - xbar_j) to row i and nothing elsewhere.
    base = _plant()
    co0 = base.coeffs.copy()
    co0[:81] = 0.0
    o0 = oracle_mod.Oracle(base.replace(coeffs=co0))
    x = W.FC9_XBAR + np.array([0.3, -0.2, 0.15, 0.05, -0.1, 0.25, 0.4, -0.35, 0.2])
    ref = o0.rhs(x, 0.9, np.zeros(9))
    for (i, j) in [(0, 8), (6, 2), (8, 0), (3, 3)]:
        co = co0.copy()
        co[9 * i + j] = 0.7
        d = oracle_mod.Oracle(base.replace(coeffs=co)).rhs(x, 0.9, np.zeros(9)) - ref
        expect = np.zeros(9)
        expect[i] = 0.7 * np.tanh(x[j] - W.FC9_XBAR[j])
        np.testing.assert_allclose(d, expect, rtol=0, atol=1e-15)


def test_fc9_closed_valve_kink(oracle_mod):
    # p_l <= p_{l+1}: q_l = 0, so row l+1 no longer depends on p_l (zero
    # derivative on that side of the kink), and at p_l = p_{l+1} the flow is 0.
    p = _special()
    o = oracle_mod.Oracle(p)
    x = np.array([2.2, 2.0, 1.8, 1.6, 1.4, 1.2, 1.1, 1.0, 1.1])
    for l in range(5):   # orifice between volumes l and l+1 (0-based)
        xa = x.copy()
        xa[l] = xa[l + 1] - 0.05
        xb = xa.copy()
        xb[l] -= 0.03
        ra, rb = o.rhs(xa, 0.5, np.zeros(9)), o.rhs(xb, 0.5, np.zeros(9))
        assert ra[l + 1] == rb[l + 1]
        xc = x.copy()
        xc[l] = xc[l + 1]
        # row l+1 = q_l - q_{l+1} with q_l = 0 at equal pressures
        k_next = p.coeffs[99 + l + 1]
        down = x[l + 2] if l + 2 < 6 else p.coeffs[111]
        assert o.rhs(xc, 0.5, np.zeros(9))[l + 1] == pytest.approx(
            -k_next * np.sqrt(xc[l + 1] - down), abs=1e-14)

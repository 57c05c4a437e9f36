"""Seeded synthetic inputs for the robust reference governor.

This module only *generates data*: plant coefficients, constraint sets,
scenario-distribution parameters and reference sequences, from fixed seeds.  It
holds none of the governor's arithmetic (no dynamics, no margins, no search), so
both the GPU library's callers and the CPU reference can consume its output
without sharing any of the method's code.

The paper benchmarks on a fuel-cell air-path model whose equations live only in
its citations (Sec. IV-A); the workloads below stand in for it:

* ``LQ4``: a 4-state linear-plus-quadratic closed loop
  ``xdot = A x + B v + G (x*x) + E w``, ``y = C x``, box ``|y_i| <= 1``.
* ``FC9``: a 9-state air-supply-like chain of volumes with square-root orifice
  flows, tanh couplings and bilinear actuator terms, 20 uncertain coefficients
  and an oxygen-excess-ratio-like lower bound (Sec. IV-A constrains OER >= 1.9).

Disturbances are uniform boxes, the structure the paper uses for its
fuel-cell simulation (Sec. IV-A: uniform per-state ranges).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

PLANT_LQ4 = 1
PLANT_FC9 = 2
INJECT_ODE = 0
INJECT_POST = 1


@dataclasses.dataclass
class Problem:
    """One RG problem: plant, constraints, scenario distribution, horizon."""

    kind: int
    n: int
    n_w: int
    n_y: int
    n_theta: int
    coeffs: np.ndarray          # float64, layout per plant kind
    F: np.ndarray               # (n_c, n_y) float64
    g: np.ndarray               # (n_c,) float64
    eps: float
    ss_check: int
    N: int
    seed: int
    instance: int
    w_lo: np.ndarray            # (n_w,)
    w_hi: np.ndarray            # (n_w,)
    theta_rel: float
    inject: int
    H: int
    dt: float

    @property
    def n_c(self) -> int:
        return int(self.F.shape[0])

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def _haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))[None, :]


def lq4_coeffs(seed: int, quad_scale: float = 0.05) -> np.ndarray:
    """A = Q diag(lambda) Q^T with lambda ~ U[-5, -0.5] and Q Haar-orthogonal;
    B ~ N(0,1) 4x1, E ~ N(0,1) 4x2, G ~ N(0, quad_scale^2) 4x4, C ~ N(0,1) 2x4.
    Layout: A[16] B[4] G[16] E[8] C[8], row-major."""
    rng = np.random.default_rng(seed)
    lam = rng.uniform(-5.0, -0.5, size=4)
    Q = _haar_orthogonal(rng, 4)
    A = Q @ np.diag(lam) @ Q.T
    B = rng.standard_normal(4)
    E = rng.standard_normal((4, 2))
    G = quad_scale * rng.standard_normal((4, 4))
    C = rng.standard_normal((2, 4))
    return np.concatenate([A.ravel(), B, G.ravel(), E.ravel(), C.ravel()]).astype(np.float64)


def lq4_problem(seed: int = 7, N: int = 64, H: int = 500, dt: float = 0.01,
                w_half: float = 0.05, eps: float = 0.05, quad_scale: float = 0.05,
                scen_seed: int = 1234, instance: int = 0, inject: int = INJECT_ODE,
                ss_check: int = 1) -> Problem:
    F = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])
    g = np.ones(4)
    return Problem(kind=PLANT_LQ4, n=4, n_w=2, n_y=2, n_theta=0,
                   coeffs=lq4_coeffs(seed, quad_scale), F=F, g=g, eps=eps, ss_check=ss_check,
                   N=N, seed=scen_seed, instance=instance,
                   w_lo=np.full(2, -w_half), w_hi=np.full(2, w_half), theta_rel=0.0,
                   inject=inject, H=H, dt=dt)


# FC9 nominal constants.  Layout: W[81] xbar[9] theta_nom[20] c_q0 p_amb d0 d1 p1ref.
# theta = (a[9], k[6], b[3], mu[2]): a slow compressor (a7 = 2) and a fast
# demand state (a9 = 12), so the supply/demand ratio y1 dips mid-transient
# after a set-point increase, by an amount that grows with the step and
# varies with the sampled coefficients.
FC9_XBAR = np.array([1.6, 1.5, 1.4, 1.3, 1.2, 1.1, 1.0, 1.0, 1.0])
FC9_THETA_NOM = np.array([3.0] * 6 + [2.0, 3.0, 12.0] + [1.0] * 6 + [1.5, 0.5, 6.0] + [0.5, 0.5])
FC9_SCALARS = np.array([0.7, 1.0, 0.05, 0.25, 1.6])  # c_q0, p_amb, d0, d1, p1ref


def fc9_coeffs(seed: int, w_scale: float = 0.3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    W = w_scale * rng.standard_normal((9, 9))
    return np.concatenate([W.ravel(), FC9_XBAR, FC9_THETA_NOM, FC9_SCALARS]).astype(np.float64)


def fc9_problem(seed: int = 11, N: int = 1024, H: int = 1000, dt: float = 0.002,
                w_half: float = 0.02, theta_rel: float = 0.1, eps: float = 0.05,
                y1_min: float = 2.35, p1_max: float = 2.1, om1_max: float = 2.2,
                scen_seed: int = 4321, instance: int = 0, inject: int = INJECT_ODE,
                ss_check: int = 1) -> Problem:
    """Outputs y = (c_q0 w1 / (d0 + d1 w3), p1, w1); constraints y1 >= y1_min,
    p1 <= p1_max, w1 <= om1_max written as F y <= g."""
    F = np.array([[-1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    g = np.array([-y1_min, p1_max, om1_max])
    return Problem(kind=PLANT_FC9, n=9, n_w=9, n_y=3, n_theta=20,
                   coeffs=fc9_coeffs(seed), F=F, g=g, eps=eps, ss_check=ss_check,
                   N=N, seed=scen_seed, instance=instance,
                   w_lo=np.full(9, -w_half), w_hi=np.full(9, w_half), theta_rel=theta_rel,
                   inject=inject, H=H, dt=dt)


def reference_sequence(seed: int, T: int, switch_every: int = 25, lo: float = -2.0,
                       hi: float = 2.0) -> np.ndarray:
    """Piecewise-constant reference: a new level ~ U[lo, hi] every `switch_every` steps."""
    rng = np.random.default_rng(seed)
    n_levels = (T + switch_every - 1) // switch_every
    levels = rng.uniform(lo, hi, size=n_levels)
    return np.repeat(levels, switch_every)[:T].astype(np.float64)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

# The LQ4 workloads use plant seed 24 and a 1 % steady-state tightening: with
# this tightening the disturbed scenario rollouts, not the steady-state test,
# decide the admissible kappa whenever the reference is not admissible (a
# 5 % tightening lets the steady-state test alone decide every step of these
# overdamped plants).
LQ4_PLANT_SEED = 24
LQ4_EPS = 0.01


def workload_lq4_fp64_single() -> dict:
    """Plain FP64 scenario RG, one update: LQ4, N=64, H=500, dt=0.01,
    x0=0, v_prev=0, r=1.5, 12 halvings."""
    p = lq4_problem(seed=LQ4_PLANT_SEED, N=64, H=500, dt=0.01, eps=LQ4_EPS)
    return dict(name="lq4_fp64_n64_h500", problem=p, x0=np.zeros(4), v_prev=0.0, r=1.5, K=12)


def workload_lq4_closed_loop(T: int = 200) -> dict:
    """FP32 rollouts with FP64 near-boundary recheck: LQ4, N=4096, H=2000,
    dt=0.005, closed loop over T RG steps tracking a piecewise-constant
    reference (levels U[-2, 2], new level every 25 steps), 12 halvings per
    step, recheck band 1e-4."""
    p = lq4_problem(seed=LQ4_PLANT_SEED, N=4096, H=2000, dt=0.005, eps=LQ4_EPS)
    return dict(name="lq4_closed_loop_n4096_h2000", problem=p, x0=np.zeros(4), v_prev=0.0,
                r_seq=reference_sequence(2024, T), K=12, band=1e-4, T=T)


@dataclasses.dataclass
class BatchInstance:
    problem: Problem
    x0: np.ndarray
    v_prev: float
    r: float


def batch_instances(count: int = 1024, seed: int = 99, n_min: int = 256, n_max: int = 8192,
                    h_min: int = 200, h_max: int = 3000, dt: float = 0.005,
                    max_count: Optional[int] = None) -> List[BatchInstance]:
    """Independent RG instances, half LQ4 and half FC9, N ~ U{n_min..n_max},
    H ~ U{h_min..h_max}, each with its own scenario seed and reference (LQ4
    instances also their own plant seed).  LQ4 instances start at x = 0 with
    v_prev = 0.  FC9 instances start with v_prev = 0.5 at the nominal
    equilibrium of that set-point (as the 9-state grid and adjoint workloads);
    their x0 is None here and the caller fills it in (all FC9 instances share
    the nominal plant, so one equilibrium serves them all)."""
    rng = np.random.default_rng(seed)
    out: List[BatchInstance] = []
    for i in range(count):
        N = int(rng.integers(n_min, n_max + 1))
        H = int(rng.integers(h_min, h_max + 1))
        if i % 2 == 0:
            p = lq4_problem(seed=int(rng.integers(1, 1 << 30)), N=N, H=H, dt=dt,
                            scen_seed=int(rng.integers(1, 1 << 31)), instance=i)
            x0 = np.zeros(4)
            r = float(rng.uniform(-2.0, 2.0))
            v_prev = 0.0
        else:
            p = fc9_problem(N=N, H=H, dt=dt, scen_seed=int(rng.integers(1, 1 << 31)), instance=i)
            x0 = None
            r = float(rng.uniform(0.5, 2.0))
            v_prev = 0.5
        out.append(BatchInstance(problem=p, x0=x0, v_prev=v_prev, r=r))
    return out


def workload_fc9_grid() -> dict:
    """FC9, N=65536 scenarios (parameters +-10 % on 20 coefficients, additive
    disturbance +-0.02), H=1000, dt=0.002, 3 output constraints; 64-point kappa
    grid evaluated in parallel, then 6 bisection refinements, FP32 rollouts with
    FP64 near-boundary recheck.  Starts at the equilibrium of v_prev = 0.5 with
    the set-point request r = 2.0 (the supply ratio dips mid-transient)."""
    p = fc9_problem(N=65536, H=1000, dt=0.002)
    return dict(name="fc9_grid_n65536_h1000", problem=p, v_prev=0.5, r=2.0, M=64, refine=6,
                band=1e-4)


def workload_fc9_adjoint() -> dict:
    """FC9, N=16384, H=1000, dt=0.002: worst-margin derivative by the reverse
    sweep with checkpoints every 50 steps, and the Newton search to 2^-12."""
    p = fc9_problem(N=16384, H=1000, dt=0.002)
    return dict(name="fc9_adjoint_n16384_h1000", problem=p, v_prev=0.5, r=2.0, Kc=50, K=12)

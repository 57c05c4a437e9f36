"""TEST INFRASTRUCTURE ONLY: Python access to the FP64 CPU reference (rg_oracle.c).

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module.  It never touches the GPU library and the GPU
library never touches it.  Problems are passed duck-typed (any object with the
fields of ``paper_2510_08288_amd.workloads.Problem``); nothing is imported from
the GPU package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rg_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

MAXN, MAXW, MAXY, MAXC, MAXTH, MAXCOEF = 9, 9, 4, 8, 20, 128


def build(force: bool = True) -> str:
    """Compile the reference with gcc: -O2, no FMA contraction, no fast-math."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-Wall",
               "-fPIC", "-shared", "-o", tmp, SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class _Problem(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("n", C.c_int32), ("n_w", C.c_int32), ("n_y", C.c_int32),
        ("n_theta", C.c_int32), ("coeffs", C.c_double * MAXCOEF), ("n_c", C.c_int32),
        ("F", C.c_double * (MAXC * MAXY)), ("g", C.c_double * MAXC), ("eps", C.c_double),
        ("ss_check", C.c_int32), ("N", C.c_int32), ("seed", C.c_uint32),
        ("instance", C.c_uint32), ("w_lo", C.c_double * MAXW), ("w_hi", C.c_double * MAXW),
        ("theta_rel", C.c_double), ("inject", C.c_int32), ("H", C.c_int32),
        ("dt", C.c_double), ("nthreads", C.c_int32),
    ]


class _Result(C.Structure):
    _fields_ = [("kappa", C.c_double), ("v", C.c_double), ("worst", C.c_double),
                ("passes", C.c_int32), ("status", C.c_int32)]


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        P = C.POINTER(_Problem)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        u32p = C.POINTER(C.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_uniform_box.argtypes = [C.c_uint32, C.c_double, C.c_double]
        L.orc_uniform_box.restype = C.c_float
        L.orc_draw_w.argtypes = [P, C.c_uint32, C.c_uint32, C.c_uint32, dp]
        L.orc_draw_theta.argtypes = [P, C.c_uint32, C.c_uint32, dp]
        L.orc_draw_true_w.argtypes = [P, C.c_uint32, dp]
        L.orc_rhs.argtypes = [P, dp, dp, C.c_double, dp, dp]
        L.orc_output.argtypes = [P, dp, C.c_double, dp]
        L.orc_rk4.argtypes = [P, dp, dp, C.c_double, dp, dp]
        L.orc_step.argtypes = [P, dp, dp, C.c_double, dp, dp]
        L.orc_margin.argtypes = [P, dp, ip]
        L.orc_margin.restype = C.c_double
        L.orc_candidate_v.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_candidate_v.restype = C.c_double
        L.orc_rollout.argtypes = [P, dp, C.c_double, C.c_uint32, C.c_uint32, ip, ip, dp]
        L.orc_rollout.restype = C.c_double
        L.orc_steady_margin.argtypes = [P, C.c_double, dp, ip]
        L.orc_steady_margin.restype = C.c_double
        L.orc_candidate.argtypes = [P, dp, C.c_double, C.c_uint32, dp, ip, dp]
        L.orc_candidate.restype = C.c_double
        L.orc_bisect.argtypes = [P, dp, C.c_double, C.c_double, C.c_uint32, C.c_int32, dp, dp]
        L.orc_bisect.restype = _Result
        L.orc_alg2.argtypes = [P, dp, C.c_double, C.c_double, C.c_uint32, C.c_int32]
        L.orc_alg2.restype = _Result
        L.orc_grid.argtypes = [P, dp, C.c_double, C.c_double, C.c_uint32, C.c_int32, C.c_int32,
                               C.POINTER(C.c_uint8)]
        L.orc_grid.restype = _Result
        L.orc_candidate_q.argtypes = [P, dp, C.c_double, C.c_uint32, C.c_int32, dp, ip]
        L.orc_candidate_q.restype = C.c_double
        L.orc_bisect_q.argtypes = [P, dp, C.c_double, C.c_double, C.c_uint32, C.c_int32,
                                   C.c_int32]
        L.orc_bisect_q.restype = _Result
        L.orc_plant_step.argtypes = [P, dp, C.c_double, C.c_uint32, dp]
        L.orc_closed_loop.argtypes = [P, dp, C.c_double, dp, C.c_int32, C.c_uint32, C.c_int32,
                                      C.c_int32, C.c_int32, C.c_int32, dp, dp, dp]
        L.orc_closed_loop.restype = C.c_int32
        L.orc_rollout_tangent.argtypes = [P, dp, C.c_double, C.c_uint32, C.c_uint32, dp, dp, ip, ip]
        L.orc_rollout_tangent.restype = C.c_double
        L.orc_steady_tangent.argtypes = [P, C.c_double, dp, dp]
        L.orc_steady_tangent.restype = C.c_double
        L.orc_candidate_grad.argtypes = [P, dp, C.c_double, C.c_double, C.c_double, C.c_uint32,
                                         dp, dp, ip]
        L.orc_candidate_grad.restype = C.c_double
        L.orc_newton.argtypes = [P, dp, C.c_double, C.c_double, C.c_uint32, C.c_int32, ip, ip]
        L.orc_newton.restype = _Result
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def problem_struct(p, nthreads: int = 1) -> _Problem:
    s = _Problem()
    s.kind, s.n, s.n_w, s.n_y, s.n_theta = p.kind, p.n, p.n_w, p.n_y, p.n_theta
    co = _f64(p.coeffs)
    assert co.size <= MAXCOEF
    for i, v in enumerate(co):
        s.coeffs[i] = float(v)
    F = _f64(p.F)
    s.n_c = F.shape[0]
    for r in range(F.shape[0]):
        for i in range(F.shape[1]):
            s.F[r * p.n_y + i] = float(F[r, i])
    for r, v in enumerate(_f64(p.g)):
        s.g[r] = float(v)
    s.eps, s.ss_check, s.N = float(p.eps), int(p.ss_check), int(p.N)
    s.seed, s.instance = int(p.seed) & 0xFFFFFFFF, int(p.instance) & 0xFFFFFFFF
    for i in range(p.n_w):
        s.w_lo[i] = float(p.w_lo[i])
        s.w_hi[i] = float(p.w_hi[i])
    s.theta_rel, s.inject, s.H, s.dt = float(p.theta_rel), int(p.inject), int(p.H), float(p.dt)
    s.nthreads = int(nthreads)
    return s


class Oracle:
    """Bound reference for one problem."""

    def __init__(self, problem, nthreads: int = 1):
        self.p = problem
        self.s = problem_struct(problem, nthreads)
        self.L = lib()

    @property
    def ref(self):
        return C.byref(self.s)

    # -- draws ----------------------------------------------------------------
    def draw_w(self, t: int, k: int, j: int) -> np.ndarray:
        w = np.zeros(MAXW)
        self.L.orc_draw_w(self.ref, t, k, j, _dp(w))
        return w[: self.p.n_w]

    def draw_theta(self, t: int, k: int) -> np.ndarray:
        th = np.zeros(MAXTH)
        self.L.orc_draw_theta(self.ref, t, k, _dp(th))
        return th[: self.p.n_theta]

    def draw_true_w(self, t: int) -> np.ndarray:
        w = np.zeros(MAXW)
        self.L.orc_draw_true_w(self.ref, t, _dp(w))
        return w[: self.p.n_w]

    # -- plant ----------------------------------------------------------------
    def rhs(self, x, v, w=None, theta=None) -> np.ndarray:
        x = _f64(x)
        w = _f64(np.zeros(MAXW) if w is None else np.pad(_f64(w), (0, MAXW - len(w))))
        out = np.zeros(MAXN)
        th = None if theta is None else _f64(theta)
        self.L.orc_rhs(self.ref, None if th is None else _dp(th), _dp(x), float(v), _dp(w), _dp(out))
        return out[: self.p.n]

    def output(self, x, v) -> np.ndarray:
        x = _f64(x)
        y = np.zeros(MAXY)
        self.L.orc_output(self.ref, _dp(x), float(v), _dp(y))
        return y[: self.p.n_y]

    def step(self, x, v, w, theta=None) -> np.ndarray:
        x = _f64(x)
        w = _f64(np.pad(_f64(w), (0, MAXW - len(w))))
        out = np.zeros(MAXN)
        th = None if theta is None else _f64(theta)
        self.L.orc_step(self.ref, None if th is None else _dp(th), _dp(x), float(v), _dp(w), _dp(out))
        return out[: self.p.n]

    def margin(self, y) -> float:
        y = _f64(y)
        return float(self.L.orc_margin(self.ref, _dp(y), None))

    # -- prediction -----------------------------------------------------------
    def rollout(self, x0, v, t, k, traj: bool = False):
        x0 = _f64(x0)
        ja, ra = C.c_int32(0), C.c_int32(0)
        tr = np.zeros((self.p.H + 1, self.p.n)) if traj else None
        m = self.L.orc_rollout(self.ref, _dp(x0), float(v), t, k, C.byref(ja), C.byref(ra),
                               None if tr is None else _dp(tr))
        if traj:
            return m, ja.value, ra.value, tr
        return m, ja.value, ra.value

    def steady_margin(self, v):
        xs = np.zeros(MAXN)
        it = C.c_int32(0)
        m = self.L.orc_steady_margin(self.ref, float(v), _dp(xs), C.byref(it))
        return m, xs[: self.p.n], it.value

    def candidate(self, x0, v, t):
        """Returns (M, per-scenario margins, argmin scenario, m_ss)."""
        x0 = _f64(x0)
        per = np.zeros(max(self.p.N, 1))
        ka = C.c_int32(0)
        mss = C.c_double(0)
        M = self.L.orc_candidate(self.ref, _dp(x0), float(v), t, _dp(per), C.byref(ka), C.byref(mss))
        return M, per[: self.p.N], ka.value, mss.value

    @staticmethod
    def candidate_v(kappa, r, v_prev) -> float:
        return float(lib().orc_candidate_v(float(kappa), float(r), float(v_prev)))

    # -- searches ---------------------------------------------------------------
    def bisect(self, x0, r, v_prev, t, K, trace: bool = False):
        x0 = _f64(x0)
        tk = np.zeros(K + 1)
        tm = np.zeros(K + 1)
        res = self.L.orc_bisect(self.ref, _dp(x0), float(r), float(v_prev), t, K, _dp(tk), _dp(tm))
        out = dict(kappa=res.kappa, v=res.v, worst=res.worst, passes=res.passes, status=res.status)
        if trace:
            out["trace_kappa"] = tk[: res.passes]
            out["trace_margin"] = tm[: res.passes]
        return out

    def alg2(self, x0, r, v_prev, t, K):
        x0 = _f64(x0)
        res = self.L.orc_alg2(self.ref, _dp(x0), float(r), float(v_prev), t, K)
        return dict(kappa=res.kappa, v=res.v, worst=res.worst, passes=res.passes, status=res.status)

    def grid(self, x0, r, v_prev, t, M, refine=0, want_P: bool = False):
        x0 = _f64(x0)
        P = np.zeros((M, max(self.p.N, 1)), dtype=np.uint8)
        res = self.L.orc_grid(self.ref, _dp(x0), float(r), float(v_prev), t, M, refine,
                              P.ctypes.data_as(C.POINTER(C.c_uint8)))
        out = dict(kappa=res.kappa, v=res.v, worst=res.worst, passes=res.passes, status=res.status)
        if want_P:
            out["P"] = P[:, : self.p.N]
        return out

    def candidate_q(self, x0, v, t, q):
        """(M_q, per-scenario margins, number of violating scenarios)."""
        x0 = _f64(x0)
        per = np.zeros(max(self.p.N, 1))
        nv = C.c_int32(0)
        M = self.L.orc_candidate_q(self.ref, _dp(x0), float(v), t, int(q), _dp(per), C.byref(nv))
        return M, per[: self.p.N], nv.value

    def bisect_q(self, x0, r, v_prev, t, K, q):
        x0 = _f64(x0)
        res = self.L.orc_bisect_q(self.ref, _dp(x0), float(r), float(v_prev), t, K, int(q))
        return dict(kappa=res.kappa, v=res.v, worst=res.worst, passes=res.passes,
                    status=res.status)

    # -- sensitivities -----------------------------------------------------------
    def rollout_tangent(self, x0, v, t, k):
        """(m, dm/dv, dm/dtheta_nom[n_theta], j*, r*) of scenario k."""
        x0 = _f64(x0)
        dv = C.c_double()
        dth = np.zeros(MAXTH)
        ja, ra = C.c_int32(), C.c_int32()
        m = self.L.orc_rollout_tangent(self.ref, _dp(x0), float(v), t, k, C.byref(dv), _dp(dth),
                                       C.byref(ja), C.byref(ra))
        return m, dv.value, dth[: self.p.n_theta], ja.value, ra.value

    def steady_tangent(self, v):
        dv = C.c_double()
        dth = np.zeros(MAXTH)
        m = self.L.orc_steady_tangent(self.ref, float(v), C.byref(dv), _dp(dth))
        return m, dv.value, dth[: self.p.n_theta]

    def candidate_grad(self, x0, kappa, r, v_prev, t):
        """(M(kappa), dM/dkappa, dM/dtheta_nom, arg-min scenario or -1 for the steady state)."""
        x0 = _f64(x0)
        dk = C.c_double()
        dth = np.zeros(MAXTH)
        ka = C.c_int32()
        M = self.L.orc_candidate_grad(self.ref, _dp(x0), float(kappa), float(r), float(v_prev), t,
                                      C.byref(dk), _dp(dth), C.byref(ka))
        return M, dk.value, dth[: self.p.n_theta], ka.value

    def newton(self, x0, r, v_prev, t, K):
        x0 = _f64(x0)
        rounds, fb = C.c_int32(), C.c_int32()
        res = self.L.orc_newton(self.ref, _dp(x0), float(r), float(v_prev), t, K, C.byref(rounds),
                                C.byref(fb))
        return dict(kappa=res.kappa, v=res.v, worst=res.worst, passes=res.passes,
                    status=res.status, rounds=rounds.value, fallbacks=fb.value)

    # -- closed loop ------------------------------------------------------------
    def plant_step(self, x, v, t) -> np.ndarray:
        x = _f64(x)
        out = np.zeros(MAXN)
        self.L.orc_plant_step(self.ref, _dp(x), float(v), t, _dp(out))
        return out[: self.p.n]

    def closed_loop(self, x0, v0, r_seq, t0=0, search="bisect", K=12, M=64, refine=0):
        r_seq = _f64(r_seq)
        T = len(r_seq)
        v = np.zeros(T)
        kap = np.zeros(T)
        xs = np.zeros((T + 1, self.p.n))
        code = {"bisect": 0, "grid": 1, "alg2": 2}[search]
        x0 = _f64(x0)
        inf = self.L.orc_closed_loop(self.ref, _dp(x0), float(v0), _dp(r_seq), T, t0, code, K, M,
                                     refine, _dp(v), _dp(kap), _dp(xs))
        return dict(v=v, kappa=kap, x=xs, infeasible_steps=inf)


def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def uniform_box(word: int, lo: float, hi: float) -> float:
    return float(lib().orc_uniform_box(int(word) & 0xFFFFFFFF, float(lo), float(hi)))

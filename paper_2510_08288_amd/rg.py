"""Python binding of librg (include/rg.h): argument marshalling only.

Every step of the governor runs in the HIP kernels of ``librg.so``.  PyTorch
supplies the device memory (the handle's workspace is a ``torch.uint8``
tensor) and the stream (``torch.cuda.current_stream()``).  If the library is
missing this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librg.so")

RG_OK = 0
RG_S_INFEASIBLE = 1
RG_S_FALLBACK = 2
RG_E_INVAL = -1
RG_E_NOMEM = -2
RG_E_HIP = -3
RG_E_NOTSUP = -4
RG_E_STATE = -5

PREC_F32_RECHECK = 0
PREC_F64 = 1
SEARCH_BISECT = 0
SEARCH_GRID = 1
SEARCH_NEWTON = 2
SEARCH_ALG2 = 3
SEARCH_NEWTON_TAN = 4
FLAG_GRID_NONMONOTONE = 1
RNG_STREAM = 0
RNG_INLINE = 1


class RGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"librg error {code}: {msg}")
        self.code = code


class rg_plant(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("n_w", C.c_int32), ("n_y", C.c_int32),
                ("n_theta", C.c_int32), ("coeffs", C.POINTER(C.c_double)), ("n_coeffs", C.c_int32)]


class rg_scenarios(C.Structure):
    _fields_ = [("N", C.c_int32), ("seed", C.c_uint32), ("instance", C.c_uint32),
                ("w_lo", C.POINTER(C.c_double)), ("w_hi", C.POINTER(C.c_double)),
                ("theta_rel", C.c_double), ("inject", C.c_int32), ("rng_mode", C.c_int32)]


class rg_constraints(C.Structure):
    _fields_ = [("n_c", C.c_int32), ("F", C.POINTER(C.c_double)), ("g", C.POINTER(C.c_double)),
                ("eps", C.c_double), ("ss_check", C.c_int32)]


class rg_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("band", C.c_double), ("K", C.c_int32),
                ("search", C.c_int32), ("depth", C.c_int32), ("M", C.c_int32),
                ("refine", C.c_int32), ("early_exit", C.c_int32), ("block", C.c_int32),
                ("max_T", C.c_int32), ("lanes", C.c_int32), ("Kc", C.c_int32),
                ("persistent_wgs", C.c_int32), ("predict", C.c_int32),
                ("speculate", C.c_int32), ("chance_q", C.c_int32)]


class rg_instance_desc(C.Structure):
    _fields_ = [("plant", rg_plant), ("scen", rg_scenarios), ("cons", rg_constraints),
                ("H", C.c_int32), ("dt", C.c_double)]


class rg_step_info(C.Structure):
    _fields_ = [("kappa", C.c_double), ("v", C.c_double), ("worst_margin", C.c_double),
                ("status", C.c_int32), ("rounds", C.c_int32), ("candidates", C.c_int32),
                ("rechecks", C.c_int32), ("bisect_passes", C.c_int32), ("t", C.c_uint32),
                ("lane_steps", C.c_uint64), ("flags", C.c_int32)]


class rg_profile(C.Structure):
    _fields_ = [("rollout_launches", C.c_int64), ("rollout_ms", C.c_double),
                ("lane_steps", C.c_uint64), ("steps", C.c_int64)]


_lib: Optional[C.CDLL] = None

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p


def load_library(path: str = LIB_PATH, with_torch: bool = True) -> C.CDLL:
    """Load librg.so.  With ``with_torch`` the HIP runtime torch already loaded is
    the one the library binds to (one runtime per process)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    if with_torch:
        import torch  # noqa: F401  (loads torch's HIP runtime first)
    L = C.CDLL(path)
    L.rg_default_options.argtypes = [C.POINTER(rg_options)]
    L.rg_create.argtypes = [C.POINTER(rg_plant), C.POINTER(rg_scenarios), C.POINTER(rg_constraints),
                            C.c_int32, C.c_double, C.POINTER(rg_options), C.POINTER(_vp)]
    L.rg_destroy.argtypes = [_vp]
    L.rg_workspace_size.argtypes = [_vp, C.POINTER(C.c_size_t)]
    L.rg_bind_workspace.argtypes = [_vp, _vp, C.c_size_t]
    L.rg_set_stream.argtypes = [_vp, _vp]
    L.rg_set_step.argtypes = [_vp, C.c_uint32]
    L.rg_reset.argtypes = [_vp]
    L.rg_get_step.argtypes = [_vp, C.POINTER(C.c_uint32)]
    L.rg_step.argtypes = [_vp, _dp, C.c_double, C.c_double, _dp, _dp, C.POINTER(rg_step_info)]
    L.rg_step_async.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.rg_step_noalloc.argtypes = [_vp, _dp, C.c_double, C.c_double, _dp, _dp,
                                  C.POINTER(rg_step_info)]
    L.rg_margin.argtypes = [_vp, _dp, C.c_double, C.c_double, _dp, C.c_int32, _dp, _fp, _ip]
    L.rg_closed_loop.argtypes = [_vp, _dp, C.c_double, _dp, C.c_int32, _dp, _dp, _dp,
                                 C.POINTER(rg_step_info), C.c_int32]
    L.rg_set_profiling.argtypes = [_vp, C.c_int32]
    L.rg_get_options.argtypes = [_vp, C.POINTER(rg_options)]
    L.rg_autotune.argtypes = [_vp, _dp, C.c_double, _dp, C.c_int32, C.c_int32,
                              C.POINTER(rg_options), C.POINTER(C.c_double)]
    L.rg_grad.argtypes = [_vp, _dp, C.c_double, C.c_double, C.c_double, _fp, _dp, _dp, _dp]
    L.rg_tangent.argtypes = [_vp, _dp, C.c_double, C.c_double, C.c_double, _fp, _fp, _ip, _dp, _dp]
    L.rg_set_theta.argtypes = [_vp, _dp]
    L.rg_equilibrium.argtypes = [_vp, C.c_double, _dp]
    L.rg_batch_create.argtypes = [C.POINTER(rg_instance_desc), C.c_int32, C.POINTER(rg_options),
                                  C.POINTER(_vp)]
    L.rg_batch_destroy.argtypes = [_vp]
    L.rg_batch_set_stream.argtypes = [_vp, _vp]
    L.rg_batch_set_step.argtypes = [_vp, C.c_int32, C.c_uint32]
    L.rg_batch_get_options.argtypes = [_vp, C.POINTER(rg_options)]
    L.rg_batch_step.argtypes = [_vp, _dp, _dp, _dp, _dp, _dp, C.POINTER(rg_step_info), C.c_int32]
    L.rg_batch_autotune.argtypes = [C.POINTER(rg_instance_desc), C.c_int32, C.POINTER(rg_options),
                                    _dp, _dp, _dp, C.POINTER(rg_options), C.POINTER(C.c_double)]
    L.rg_batch_last_error.argtypes = [_vp]
    L.rg_batch_last_error.restype = C.c_char_p
    L.rg_get_profile.argtypes = [_vp, C.POINTER(rg_profile)]
    L.rg_draws.argtypes = [_vp, C.c_uint32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _fp, _dp]
    L.rg_trajectory.argtypes = [_vp, _dp, C.c_double, _ip, C.c_int32, C.c_int32, _dp]
    L.rg_fp64_tanh.argtypes = [_dp, _dp, C.c_int32]
    L.rg_status_string.argtypes = [C.c_int]
    L.rg_status_string.restype = C.c_char_p
    L.rg_last_error.argtypes = [_vp]
    L.rg_last_error.restype = C.c_char_p
    _lib = L
    return L


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray, t=_dp):
    return a.ctypes.data_as(t)


def _info_dict(info: rg_step_info) -> dict:
    return dict(worst=info.worst_margin, rounds=info.rounds, candidates=info.candidates,
                rechecks=info.rechecks, bisect_passes=info.bisect_passes, t=info.t,
                lane_steps=info.lane_steps, flags=info.flags)


def fp64_tanh(x) -> np.ndarray:
    """rg_fp64_tanh: the device FP64 tanh of the 9-state plant's FP64 paths."""
    L = load_library()
    x = _f64(np.asarray(x).reshape(-1))
    y = np.zeros_like(x)
    rc = L.rg_fp64_tanh(_ptr(x), _ptr(y), x.size)
    if rc < 0:
        raise RGError(rc, L.rg_last_error(None).decode())
    return y


def default_options() -> rg_options:
    o = rg_options()
    load_library().rg_default_options(C.byref(o))
    return o


class Governor:
    """One robust reference governor handle on the current CUDA (HIP) device."""

    def __init__(self, problem, precision: int = PREC_F32_RECHECK, band: float = 1e-4,
                 K: int = 12, search: int = SEARCH_BISECT, depth: int = 0, M: int = 64,
                 refine: int = 6, early_exit: bool = True, block: int = 0, max_T: int = 256,
                 rng_mode: int = RNG_STREAM, lanes: int = 0, Kc: int = 50,
                 predict: bool = True, speculate: int = 7, chance_q: int = 0,
                 torch_workspace: bool = True):
        import torch
        self.L = load_library()
        self.problem = problem
        p = problem
        self._coeffs = _f64(p.coeffs)
        self._wlo = _f64(p.w_lo)
        self._whi = _f64(p.w_hi)
        self._F = _f64(np.asarray(p.F).reshape(-1))
        self._g = _f64(p.g)
        plant = rg_plant(p.kind, p.n, p.n_w, p.n_y, p.n_theta, _ptr(self._coeffs), self._coeffs.size)
        scen = rg_scenarios(int(p.N), int(p.seed) & 0xFFFFFFFF, int(p.instance) & 0xFFFFFFFF,
                            _ptr(self._wlo), _ptr(self._whi), float(p.theta_rel), int(p.inject),
                            int(rng_mode))
        cons = rg_constraints(int(np.asarray(p.F).shape[0]), _ptr(self._F), _ptr(self._g),
                              float(p.eps), int(p.ss_check))
        opt = default_options()
        opt.precision, opt.band, opt.K, opt.search = precision, band, K, search
        opt.depth, opt.M, opt.refine = depth, M, refine
        opt.early_exit, opt.block, opt.max_T, opt.lanes = int(early_exit), block, max_T, lanes
        opt.Kc = Kc
        opt.predict = int(predict)
        opt.speculate = int(speculate)
        opt.chance_q = int(chance_q)
        h = _vp()
        rc = self.L.rg_create(C.byref(plant), C.byref(scen), C.byref(cons), int(p.H), float(p.dt),
                              C.byref(opt), C.byref(h))
        if rc < 0:
            raise RGError(rc, self.L.rg_last_error(None).decode())
        self.h = h
        self.options = rg_options()
        self._check(self.L.rg_get_options(self.h, C.byref(self.options)))
        self.workspace = None
        if torch_workspace:
            nbytes = C.c_size_t()
            self._check(self.L.rg_workspace_size(self.h, C.byref(nbytes)))
            # 256-byte alignment: torch's allocator returns at least 512-byte aligned blocks.
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
            self._check(self.L.rg_bind_workspace(self.h, C.c_void_p(self.workspace.data_ptr()),
                                                 int(nbytes.value)))
        # A stream of the handle's own (default priority): graph capture is not
        # allowed on the null stream.
        self.stream = torch.cuda.Stream()
        self.set_stream(self.stream)

    # -- plumbing --------------------------------------------------------------
    def _check(self, rc: int) -> int:
        if rc < 0:
            raise RGError(rc, self.L.rg_last_error(self.h).decode())
        return rc

    def set_stream(self, stream) -> None:
        handle = stream.cuda_stream if stream is not None else 0
        self._check(self.L.rg_set_stream(self.h, C.c_void_p(handle)))

    def set_step(self, t: int) -> None:
        self._check(self.L.rg_set_step(self.h, int(t)))

    def reset(self) -> None:
        """Clear the search state earlier steps left (rg_reset)."""
        self._check(self.L.rg_reset(self.h))

    def get_step(self) -> int:
        t = C.c_uint32()
        self._check(self.L.rg_get_step(self.h, C.byref(t)))
        return int(t.value)

    def close(self) -> None:
        if getattr(self, "h", None):
            self.L.rg_destroy(self.h)
            self.h = None
        self.workspace = None  # the handle is gone: its device memory may go too

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- governor ----------------------------------------------------------------
    def step(self, x, r: float, v_prev: float) -> dict:
        x = _f64(x)
        v = C.c_double()
        kap = C.c_double()
        info = rg_step_info()
        rc = self._check(self.L.rg_step(self.h, _ptr(x), float(r), float(v_prev), C.byref(v),
                                        C.byref(kap), C.byref(info)))
        return dict(v=v.value, kappa=kap.value, status=rc, **_info_dict(info))

    def step_async(self, x, r, v_prev, t, v_out, kappa_out=None, status_out=None) -> None:
        """rg_step_async: one RG step on device tensors, enqueued on the handle's
        stream (set_stream) without waiting; capturable in a CUDA graph.  x: n
        float64, r, v_prev, v_out, kappa_out: one float64 each, t: one int32
        holding the step index as uint32 (advanced by one), status_out: one
        int32; all contiguous on the handle's device."""
        n = self.problem.n
        spec = [(x, "float64", n, "x"), (r, "float64", 1, "r"), (v_prev, "float64", 1, "v_prev"),
                (t, "int32", 1, "t"), (v_out, "float64", 1, "v_out"),
                (kappa_out, "float64", 1, "kappa_out"), (status_out, "int32", 1, "status_out")]
        ptrs = []
        for a, dt, numel, name in spec:
            if a is None and name in ("kappa_out", "status_out"):
                ptrs.append(None)
                continue
            if (not a.is_cuda or str(a.dtype) != "torch." + dt or a.numel() != numel
                    or not a.is_contiguous()):
                raise ValueError(f"{name}: a contiguous {dt} device tensor of {numel} element(s)")
            ptrs.append(C.c_void_p(a.data_ptr()))
        self._check(self.L.rg_step_async(self.h, *ptrs))

    def step_noalloc(self, x, r: float, v_prev: float) -> dict:
        """rg_step_noalloc: the same RG step with no device allocation (static
        device scratch, draws regenerated in the kernels)."""
        x = _f64(x)
        v = C.c_double()
        kap = C.c_double()
        info = rg_step_info()
        rc = self._check(self.L.rg_step_noalloc(self.h, _ptr(x), float(r), float(v_prev),
                                                C.byref(v), C.byref(kap), C.byref(info)))
        return dict(v=v.value, kappa=kap.value, status=rc, **_info_dict(info))

    def margin(self, x, r: float, v_prev: float, kappas: Sequence[float],
               per_scenario: bool = False) -> dict:
        x = _f64(x)
        k = _f64(kappas)
        M = k.size
        out = np.zeros(M)
        per = np.zeros((M, self.problem.N), dtype=np.float32) if per_scenario else None
        perj = np.zeros((M, self.problem.N), dtype=np.int32) if per_scenario else None
        self._check(self.L.rg_margin(self.h, _ptr(x), float(r), float(v_prev), _ptr(k), M, _ptr(out),
                                     None if per is None else _ptr(per, _fp),
                                     None if perj is None else _ptr(perj, _ip)))
        return dict(margins=out, per_scenario=per, per_scenario_j=perj)

    def grad(self, x, r: float, v_prev: float, kappa: float, upstream=None) -> dict:
        """dM/dkappa and dM/dtheta_nom (upstream None), or the upstream-weighted sum
        of the per-scenario margin derivatives."""
        x = _f64(x)
        up = None
        if upstream is not None:
            up = np.ascontiguousarray(np.asarray(upstream, dtype=np.float32).reshape(-1))
            assert up.size == self.problem.N
        M = C.c_double()
        dk = C.c_double()
        dth = np.zeros(max(self.problem.n_theta, 1))
        self._check(self.L.rg_grad(self.h, _ptr(x), float(r), float(v_prev), float(kappa),
                                   None if up is None else _ptr(up, _fp), C.byref(M), C.byref(dk),
                                   _ptr(dth)))
        return dict(M=M.value, dkappa=dk.value, dtheta=dth[: self.problem.n_theta])

    def tangent(self, x, r: float, v_prev: float, kappa: float) -> dict:
        """rg_tangent: per-scenario FP32 margins, their forward-mode dm/dv and
        minimising steps, M(kappa) and dM/dkappa."""
        x = _f64(x)
        N = self.problem.N
        m = np.zeros(N, dtype=np.float32)
        dv = np.zeros(N, dtype=np.float32)
        j = np.zeros(N, dtype=np.int32)
        M = C.c_double()
        dk = C.c_double()
        self._check(self.L.rg_tangent(self.h, _ptr(x), float(r), float(v_prev), float(kappa),
                                      _ptr(m, _fp), _ptr(dv, _fp), _ptr(j, _ip), C.byref(M),
                                      C.byref(dk)))
        return dict(m=m, dm_dv=dv, j=j, M=M.value, dkappa=dk.value)

    def autotune(self, x0, v0: float, r_seq, apply: bool = True) -> dict:
        """Time the closed loop over r_seq under each launch schedule (rg_autotune);
        with apply the handle keeps the fastest.  Returns that schedule."""
        x0 = _f64(x0)
        r = _f64(r_seq)
        best = rg_options()
        ms = C.c_double()
        self._check(self.L.rg_autotune(self.h, _ptr(x0), float(v0), _ptr(r), r.size, int(apply),
                                       C.byref(best), C.byref(ms)))
        self.options = rg_options()
        self.L.rg_get_options(self.h, C.byref(self.options))
        return dict(lanes=best.lanes, block=best.block, depth=best.depth, predict=best.predict,
                    speculate=best.speculate, ms_per_update=ms.value)

    def equilibrium(self, v: float) -> np.ndarray:
        x = np.zeros(self.problem.n)
        self._check(self.L.rg_equilibrium(self.h, float(v), _ptr(x)))
        return x

    def set_theta(self, theta_nom) -> None:
        th = _f64(theta_nom)
        assert th.size == self.problem.n_theta
        self._check(self.L.rg_set_theta(self.h, _ptr(th)))

    def closed_loop(self, x0, v0: float, r_seq, use_graph: bool = True) -> dict:
        x0 = _f64(x0)
        r = _f64(r_seq)
        T = r.size
        v = np.zeros(T)
        kap = np.zeros(T)
        xs = np.zeros((T + 1, self.problem.n))
        infos = (rg_step_info * T)()
        self._check(self.L.rg_closed_loop(self.h, _ptr(x0), float(v0), _ptr(r), T, _ptr(v),
                                          _ptr(kap), _ptr(xs), infos, int(use_graph)))
        keys = ["status", "rounds", "candidates", "rechecks", "bisect_passes", "lane_steps", "t",
                "flags"]
        out = {k: np.array([getattr(infos[i], k) for i in range(T)]) for k in keys}
        out["worst"] = np.array([infos[i].worst_margin for i in range(T)])
        out.update(v=v, kappa=kap, x=xs)
        return out

    def set_profiling(self, enable: bool) -> None:
        self._check(self.L.rg_set_profiling(self.h, int(enable)))

    def profile(self) -> dict:
        p = rg_profile()
        self._check(self.L.rg_get_profile(self.h, C.byref(p)))
        return dict(rollout_launches=p.rollout_launches, rollout_ms=p.rollout_ms,
                    lane_steps=p.lane_steps, steps=p.steps)

    def draws(self, t: int, k0: int, nk: int, j0: int, nj: int, theta: bool = False):
        w = np.zeros((nj, nk, self.problem.n_w), dtype=np.float32)
        th = np.zeros((nk, max(self.problem.n_theta, 1))) if theta else None
        self._check(self.L.rg_draws(self.h, int(t), k0, nk, j0, nj, _ptr(w, _fp),
                                    None if th is None else _ptr(th)))
        return (w, th[:, : self.problem.n_theta]) if theta else w

    def trajectory(self, x, v: float, k_list, precision: int = PREC_F32_RECHECK) -> np.ndarray:
        x = _f64(x)
        ks = np.ascontiguousarray(np.asarray(k_list, dtype=np.int32))
        out = np.zeros((ks.size, self.problem.H + 1, self.problem.n))
        self._check(self.L.rg_trajectory(self.h, _ptr(x), float(v), _ptr(ks, _ip), ks.size,
                                         int(precision), _ptr(out)))
        return out


def _batch_descs(problems):
    """Instance descriptors of a batch, and the arrays they point into (keep them alive)."""
    keep = []
    descs = (rg_instance_desc * len(problems))()
    for i, p in enumerate(problems):
        co, wlo, whi = _f64(p.coeffs), _f64(p.w_lo), _f64(p.w_hi)
        F, g = _f64(np.asarray(p.F).reshape(-1)), _f64(p.g)
        keep += [co, wlo, whi, F, g]
        descs[i].plant = rg_plant(p.kind, p.n, p.n_w, p.n_y, p.n_theta, _ptr(co), co.size)
        descs[i].scen = rg_scenarios(int(p.N), int(p.seed) & 0xFFFFFFFF,
                                     int(p.instance) & 0xFFFFFFFF, _ptr(wlo), _ptr(whi),
                                     float(p.theta_rel), int(p.inject), RNG_INLINE)
        descs[i].cons = rg_constraints(int(np.asarray(p.F).shape[0]), _ptr(F), _ptr(g),
                                       float(p.eps), int(p.ss_check))
        descs[i].H = int(p.H)
        descs[i].dt = float(p.dt)
    return descs, keep


def _batch_options(K, band, depth, block, persistent_wgs, early_exit, predict, search, M, refine):
    opt = default_options()
    opt.K, opt.band, opt.depth, opt.block = K, band, depth, block if block else 64
    opt.persistent_wgs, opt.early_exit = persistent_wgs, int(early_exit)
    opt.predict, opt.search, opt.M, opt.refine = int(predict), search, M, refine
    return opt


def batch_autotune(problems, xs, r, v_prev, K: int = 12, band: float = 1e-4,
                   early_exit: bool = True, search: int = SEARCH_BISECT, M: int = 64,
                   refine: int = 6) -> dict:
    """rg_batch_autotune: time steps 0..2 of the batch under every schedule
    (scenario tile, depth, first-round prediction) and return the fastest one
    (keyword arguments of Batch) with its time per batched step."""
    L = load_library()
    descs, keep = _batch_descs(problems)
    opt = _batch_options(K, band, 0, 64, 0, early_exit, False, search, M, refine)
    x = _f64(np.concatenate([np.asarray(v, dtype=np.float64) for v in xs]))
    r = _f64(r)
    vp = _f64(v_prev)
    best = rg_options()
    ms = C.c_double()
    rc = L.rg_batch_autotune(descs, len(problems), C.byref(opt), _ptr(x), _ptr(r), _ptr(vp),
                             C.byref(best), C.byref(ms))
    if rc < 0:
        raise RGError(rc, L.rg_batch_last_error(None).decode())
    return dict(block=best.block, depth=best.depth, predict=bool(best.predict),
                ms_per_batched_step=ms.value)


class Batch:
    """Many independent governors stepped together (``rg_batch_*``)."""

    def __init__(self, problems, K: int = 12, band: float = 1e-4, depth: int = 0, block: int = 0,
                 persistent_wgs: int = 0, early_exit: bool = True, predict: bool = False,
                 search: int = SEARCH_BISECT, M: int = 64, refine: int = 6):
        import torch
        self.L = load_library()
        self.problems = list(problems)
        descs, self._keep = _batch_descs(self.problems)
        opt = _batch_options(K, band, depth, block, persistent_wgs, early_exit, predict, search,
                             M, refine)
        h = _vp()
        rc = self.L.rg_batch_create(descs, len(self.problems), C.byref(opt), C.byref(h))
        if rc < 0:
            raise RGError(rc, self.L.rg_batch_last_error(None).decode())
        self.h = h
        self.options = rg_options()
        self.L.rg_batch_get_options(self.h, C.byref(self.options))
        self.stream = torch.cuda.Stream()
        self._check(self.L.rg_batch_set_stream(self.h, C.c_void_p(self.stream.cuda_stream)))

    def _check(self, rc: int) -> int:
        if rc < 0:
            raise RGError(rc, self.L.rg_batch_last_error(self.h).decode())
        return rc

    def set_step(self, i: int, t: int) -> None:
        self._check(self.L.rg_batch_set_step(self.h, i, int(t)))

    def step(self, xs, r, v_prev, use_graph: bool = True) -> dict:
        x = _f64(np.concatenate([np.asarray(v, dtype=np.float64) for v in xs]))
        r = _f64(r)
        vp = _f64(v_prev)
        n = len(self.problems)
        v = np.zeros(n)
        kap = np.zeros(n)
        infos = (rg_step_info * n)()
        self._check(self.L.rg_batch_step(self.h, _ptr(x), _ptr(r), _ptr(vp), _ptr(v), _ptr(kap),
                                         infos, int(use_graph)))
        out = {k: np.array([getattr(infos[i], k) for i in range(n)])
               for k in ["status", "rounds", "candidates", "bisect_passes", "lane_steps", "t"]}
        out.update(v=v, kappa=kap)
        return out

    def close(self) -> None:
        if getattr(self, "h", None):
            self.L.rg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

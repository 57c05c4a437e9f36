"""C ABI checks that need no GPU: the library loads, exports every entry point
declared in include/rg.h, and validates arguments on the host before any
device work (rg_create allocates no device memory)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2510_08288_amd import rg as R
from paper_2510_08288_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rg_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(R.LIB_PATH):
        pytest.skip("librg.so not built")
    return R.load_library(with_torch=False)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["rg_create", "rg_destroy", "rg_step", "rg_margin", "rg_closed_loop",
                     "rg_workspace_size", "rg_bind_workspace", "rg_set_stream", "rg_set_step",
                     "rg_get_step", "rg_draws", "rg_trajectory", "rg_status_string",
                     "rg_last_error", "rg_default_options", "rg_grad", "rg_set_theta",
                     "rg_get_options", "rg_set_profiling", "rg_get_profile", "rg_autotune",
                     "rg_batch_autotune", "rg_step_async"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in [0, 1, 2, -1, -2, -3, -4, -5]:
        assert len(lib.rg_status_string(code)) > 0


def test_default_options(lib):
    o = R.rg_options()
    assert lib.rg_default_options(C.byref(o)) == 0
    assert o.K == 12 and o.band == 1e-4 and o.precision == 0 and o.early_exit == 1
    assert o.predict == 1
    assert o.speculate == 7
    assert lib.rg_default_options(None) == R.RG_E_INVAL


def _descriptors(p, **over):
    co = np.ascontiguousarray(p.coeffs, dtype=np.float64)
    wlo = np.ascontiguousarray(p.w_lo, dtype=np.float64)
    whi = np.ascontiguousarray(p.w_hi, dtype=np.float64)
    F = np.ascontiguousarray(np.asarray(p.F).reshape(-1), dtype=np.float64)
    g = np.ascontiguousarray(p.g, dtype=np.float64)
    keep = [co, wlo, whi, F, g]
    dp = C.POINTER(C.c_double)
    plant = R.rg_plant(over.get("kind", p.kind), over.get("n", p.n), p.n_w, p.n_y, p.n_theta,
                       co.ctypes.data_as(dp), over.get("n_coeffs", co.size))
    scen = R.rg_scenarios(over.get("N", p.N), p.seed, 0, wlo.ctypes.data_as(dp),
                          whi.ctypes.data_as(dp), over.get("theta_rel", p.theta_rel),
                          over.get("inject", 0), 0)
    cons = R.rg_constraints(over.get("n_c", np.asarray(p.F).shape[0]), F.ctypes.data_as(dp),
                            g.ctypes.data_as(dp), over.get("eps", p.eps), 1)
    return plant, scen, cons, keep


def _create(lib, p, H=None, dt=None, opt=None, **over):
    plant, scen, cons, keep = _descriptors(p, **over)
    h = C.c_void_p()
    rc = lib.rg_create(C.byref(plant), C.byref(scen), C.byref(cons), H or p.H, dt or p.dt,
                       None if opt is None else C.byref(opt), C.byref(h))
    return rc, h


def test_create_and_destroy_without_device(lib):
    p = W.lq4_problem(N=100, H=50)
    rc, h = _create(lib, p)
    assert rc == 0 and h.value
    size = C.c_size_t()
    assert lib.rg_workspace_size(h, C.byref(size)) == 0
    # draws buffer (H * n_w * N floats) is part of the workspace
    assert size.value >= 50 * 2 * 100 * 4
    t = C.c_uint32()
    assert lib.rg_set_step(h, 17) == 0 and lib.rg_get_step(h, C.byref(t)) == 0 and t.value == 17
    assert lib.rg_destroy(h) == 0
    assert lib.rg_destroy(None) == 0


@pytest.mark.parametrize("override,code", [
    (dict(kind=3), R.RG_E_INVAL),
    (dict(n=5), R.RG_E_INVAL),
    (dict(n_coeffs=51), R.RG_E_INVAL),
    (dict(N=0), R.RG_E_INVAL),
    (dict(theta_rel=1.5), R.RG_E_INVAL),
    (dict(inject=7), R.RG_E_INVAL),
    (dict(n_c=0), R.RG_E_INVAL),
    (dict(n_c=5), R.RG_E_NOTSUP),
    (dict(eps=1.0), R.RG_E_INVAL),
])
def test_create_rejects_bad_descriptors(lib, override, code):
    p = W.lq4_problem(N=16, H=10)
    rc, h = _create(lib, p, **override)
    assert rc == code and not h.value
    assert len(lib.rg_last_error(None)) > 0


def test_create_rejects_bad_horizon_and_options(lib):
    p = W.lq4_problem(N=16, H=10)
    assert _create(lib, p, H=-1)[0] == R.RG_E_INVAL
    assert _create(lib, p, dt=-0.1)[0] == R.RG_E_INVAL
    assert _create(lib, p, dt=float("nan"))[0] == R.RG_E_INVAL
    for field, value, code in [("K", -1, R.RG_E_INVAL), ("depth", 9, R.RG_E_INVAL),
                               ("block", 100, R.RG_E_INVAL), ("block", 512, R.RG_E_INVAL),
                               ("precision", 4, R.RG_E_INVAL), ("search", 5, R.RG_E_INVAL),
                               ("Kc", 0, R.RG_E_INVAL), ("lanes", 2, R.RG_E_INVAL), ("predict", 2, R.RG_E_INVAL),
                               ("speculate", 8, R.RG_E_INVAL),
                               ("band", float("inf"), R.RG_E_INVAL), ("max_T", 0, R.RG_E_INVAL)]:
        o = R.rg_options()
        lib.rg_default_options(C.byref(o))
        setattr(o, field, value)
        assert _create(lib, p, opt=o)[0] == code, field
    o = R.rg_options()
    lib.rg_default_options(C.byref(o))
    o.search, o.M = 1, 200
    assert _create(lib, p, opt=o)[0] == R.RG_E_INVAL
    o = R.rg_options()
    lib.rg_default_options(C.byref(o))
    o.search, o.precision = 2, 1      # Newton runs on the FP32 rollouts and adjoint only
    assert _create(lib, p, opt=o)[0] == R.RG_E_NOTSUP
    o.precision = 0
    rc, h = _create(lib, p, opt=o)
    assert rc == 0 and lib.rg_destroy(h) == 0
    # Alg. 2 tabulates the steady state of 2^K tree nodes (K <= 16) and bisects
    # each scenario on the robust verdict
    o = R.rg_options()
    lib.rg_default_options(C.byref(o))
    o.search, o.K = R.SEARCH_ALG2, 17
    assert _create(lib, p, opt=o)[0] == R.RG_E_NOTSUP
    o.K, o.chance_q = 16, 2
    assert _create(lib, p, opt=o)[0] == R.RG_E_NOTSUP
    o.chance_q = 0
    rc, h = _create(lib, p, opt=o)
    assert rc == 0
    dp = C.POINTER(C.c_double)
    x, r, v = np.zeros(4), np.zeros(3), np.zeros(3)
    assert lib.rg_closed_loop(h, x.ctypes.data_as(dp), 0.0, r.ctypes.data_as(dp), 3,
                              v.ctypes.data_as(dp), None, None, None, 0) == R.RG_E_NOTSUP
    assert lib.rg_autotune(h, x.ctypes.data_as(dp), 0.0, r.ctypes.data_as(dp), 3, 1, None,
                           None) == R.RG_E_NOTSUP
    vp = C.c_void_p(x.ctypes.data)  # refused before any pointer is read
    assert lib.rg_step_async(h, vp, vp, vp, vp, vp, None, None) == R.RG_E_NOTSUP
    assert lib.rg_destroy(h) == 0


def test_create_rejects_nonfinite_data(lib):
    p = W.lq4_problem(N=16, H=10)
    q = p.replace(coeffs=p.coeffs.copy())
    q.coeffs[3] = np.nan
    assert _create(lib, q)[0] == R.RG_E_INVAL
    q = p.replace(w_lo=np.array([0.1, 0.0]), w_hi=np.array([0.0, 0.0]))
    assert _create(lib, q)[0] == R.RG_E_INVAL


def test_calls_reject_bad_arguments_before_device_work(lib):
    p = W.lq4_problem(N=16, H=10)
    rc, h = _create(lib, p)
    assert rc == 0
    dp = C.POINTER(C.c_double)
    x = np.zeros(4)
    xn = np.array([0.0, np.nan, 0.0, 0.0])
    v = C.c_double()
    assert lib.rg_step(None, x.ctypes.data_as(dp), 1.0, 0.0, C.byref(v), None, None) == R.RG_E_INVAL
    assert lib.rg_step(h, None, 1.0, 0.0, C.byref(v), None, None) == R.RG_E_INVAL
    assert lib.rg_step(h, xn.ctypes.data_as(dp), 1.0, 0.0, C.byref(v), None, None) == R.RG_E_INVAL
    assert lib.rg_step(h, x.ctypes.data_as(dp), float("inf"), 0.0, C.byref(v), None, None) == R.RG_E_INVAL
    # the asynchronous step rejects null handles and pointers before reading any
    # of them (its pointers are device memory; these are never dereferenced)
    vp = C.c_void_p(x.ctypes.data)
    assert lib.rg_step_async(None, vp, vp, vp, vp, vp, None, None) == R.RG_E_INVAL
    assert lib.rg_step_async(h, None, vp, vp, vp, vp, None, None) == R.RG_E_INVAL
    assert lib.rg_step_async(h, vp, vp, vp, None, vp, None, None) == R.RG_E_INVAL
    assert lib.rg_step_async(h, vp, vp, vp, vp, None, None, None) == R.RG_E_INVAL
    assert b"NULL" in lib.rg_last_error(h)
    kap = np.array([0.5, 1.5])
    out = np.zeros(2)
    assert lib.rg_margin(h, x.ctypes.data_as(dp), 1.0, 0.0, kap.ctypes.data_as(dp), 2,
                         out.ctypes.data_as(dp), None, None) == R.RG_E_INVAL
    assert b"kappa" in lib.rg_last_error(h)
    dk = C.c_double()
    assert lib.rg_grad(h, x.ctypes.data_as(dp), 1.0, 0.0, 1.5, None, None, C.byref(dk), None) == R.RG_E_INVAL
    assert lib.rg_set_theta(h, x.ctypes.data_as(dp)) == R.RG_E_NOTSUP   # LQ4 has no theta
    r = np.zeros(3)
    assert lib.rg_closed_loop(h, x.ctypes.data_as(dp), 0.0, r.ctypes.data_as(dp), 0,
                              out.ctypes.data_as(dp), None, None, None, 0) == R.RG_E_INVAL
    ks = np.array([0, 99], dtype=np.int32)
    tr = np.zeros(100)
    assert lib.rg_trajectory(h, x.ctypes.data_as(dp), 0.5, ks.ctypes.data_as(C.POINTER(C.c_int32)),
                             2, 0, tr.ctypes.data_as(dp)) == R.RG_E_INVAL
    assert lib.rg_autotune(h, None, 0.0, r.ctypes.data_as(dp), 3, 1, None, None) == R.RG_E_INVAL
    assert lib.rg_autotune(h, x.ctypes.data_as(dp), 0.0, r.ctypes.data_as(dp), 0, 1, None,
                           None) == R.RG_E_INVAL
    assert lib.rg_autotune(None, x.ctypes.data_as(dp), 0.0, r.ctypes.data_as(dp), 3, 1, None,
                           None) == R.RG_E_INVAL
    assert lib.rg_bind_workspace(h, C.c_void_p(0x1001), 1 << 30) == R.RG_E_INVAL
    assert lib.rg_bind_workspace(h, C.c_void_p(0x1000), 16) == R.RG_E_NOMEM
    assert lib.rg_destroy(h) == 0


def test_batch_create_and_step_validate_on_the_host(lib):
    ps = [W.lq4_problem(N=40, H=20), W.fc9_problem(N=30, H=10)]
    descs = (R.rg_instance_desc * 2)()
    keep = []
    for i, p in enumerate(ps):
        plant, scen, cons, k = _descriptors(p)
        keep += k
        descs[i].plant, descs[i].scen, descs[i].cons = plant, scen, cons
        descs[i].H, descs[i].dt = p.H, p.dt
    h = C.c_void_p()
    assert lib.rg_batch_create(descs, 2, None, C.byref(h)) == 0 and h.value
    o = R.rg_options()
    assert lib.rg_batch_get_options(h, C.byref(o)) == 0 and 1 <= o.depth <= 6
    dp = C.POINTER(C.c_double)
    x = np.concatenate([np.zeros(4), np.asarray(W.FC9_XBAR)])
    r = np.array([1.0, 1.0])
    vp = np.zeros(2)
    v = np.zeros(2)
    xn = x.copy()
    xn[5] = np.nan
    assert lib.rg_batch_step(h, xn.ctypes.data_as(dp), r.ctypes.data_as(dp), vp.ctypes.data_as(dp),
                             v.ctypes.data_as(dp), None, None, 0) == R.RG_E_INVAL
    assert lib.rg_batch_step(h, x.ctypes.data_as(dp), None, vp.ctypes.data_as(dp),
                             v.ctypes.data_as(dp), None, None, 0) == R.RG_E_INVAL
    assert lib.rg_batch_set_step(h, 2, 5) == R.RG_E_INVAL   # two instances
    assert lib.rg_batch_destroy(h) == 0
    # the batch autotuner checks its arguments before it creates any batch
    assert lib.rg_batch_autotune(None, 2, None, x.ctypes.data_as(dp), r.ctypes.data_as(dp),
                                 vp.ctypes.data_as(dp), None, None) == R.RG_E_INVAL
    assert lib.rg_batch_autotune(descs, 2, None, x.ctypes.data_as(dp), None,
                                 vp.ctypes.data_as(dp), None, None) == R.RG_E_INVAL
    assert lib.rg_batch_autotune(descs, 0, None, x.ctypes.data_as(dp), r.ctypes.data_as(dp),
                                 vp.ctypes.data_as(dp), None, None) == R.RG_E_INVAL
    # Newton, Alg. 2 and the chance-constrained verdict are not batched
    for field, value in [("search", R.SEARCH_NEWTON), ("search", R.SEARCH_ALG2), ("chance_q", 3)]:
        o = R.rg_options()
        lib.rg_default_options(C.byref(o))
        setattr(o, field, value)
        h3 = C.c_void_p()
        assert lib.rg_batch_create(descs, 2, C.byref(o), C.byref(h3)) == R.RG_E_NOTSUP
    descs[1].scen.N = 0
    h2 = C.c_void_p()
    assert lib.rg_batch_create(descs, 2, None, C.byref(h2)) == R.RG_E_INVAL
    assert b"instance 1" in lib.rg_batch_last_error(None)
    # an invalid descriptor fails in the autotuner's first rg_batch_create
    assert lib.rg_batch_autotune(descs, 2, None, x.ctypes.data_as(dp), r.ctypes.data_as(dp),
                                 vp.ctypes.data_as(dp), None, None) == R.RG_E_INVAL
    assert b"instance 1" in lib.rg_batch_last_error(None)


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C layout (sizes and
    every field offset, from a host C program compiled against include/rg.h)."""
    import subprocess
    structs = {"rg_plant": R.rg_plant, "rg_scenarios": R.rg_scenarios,
               "rg_constraints": R.rg_constraints, "rg_options": R.rg_options,
               "rg_step_info": R.rg_step_info, "rg_profile": R.rg_profile,
               "rg_instance_desc": R.rg_instance_desc}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rg.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for ln in filter(None, out):
        name, field, value = ln.split()
        cls = structs[name]
        if field == "size":
            assert C.sizeof(cls) == int(value), name
        else:
            assert getattr(cls, field).offset == int(value), (name, field)

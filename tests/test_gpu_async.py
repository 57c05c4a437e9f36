"""GPU tests of rg_step_async, the RG step on device pointers: the same kappa,
v and status as rg_step at every step of a sequence (bisection, grid, both
Newton forms, FP32 with FP64 recheck and plain FP64, both plants, the
chance-constrained verdict), the device step counter advanced in
place, and a CUDA graph captured around one step and replayed several times,
with eager work and synchronisation between the replays, every replay checked
against rg_step."""
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


def _dev(torch):
    f64 = dict(dtype=torch.float64, device="cuda")
    i32 = dict(dtype=torch.int32, device="cuda")
    return dict(r=torch.zeros(1, **f64), vp=torch.zeros(1, **f64), v=torch.zeros(1, **f64),
                k=torch.zeros(1, **f64), t=torch.zeros(1, **i32), st=torch.zeros(1, **i32))


def _states(R, p, g, r_seq):
    # start states near the equilibria of the references (a steady start for
    # the 9-state plant, whose zero state is far from any)
    rng = np.random.default_rng(3)
    return [g.equilibrium(float(r)) + 0.02 * rng.standard_normal(p.n) for r in r_seq]


CASES = {
    "lq4_bisect": (lambda: W.lq4_problem(seed=24, N=512, H=400, dt=0.005, eps=0.01), {}),
    "lq4_bisect_inline": (lambda: W.lq4_problem(seed=24, N=300, H=300, dt=0.005, eps=0.01),
                          dict(rng_mode=1)),
    "lq4_newton": (lambda: W.lq4_problem(seed=24, N=256, H=300, dt=0.005, eps=0.01),
                   dict(search=2)),
    "lq4_newton_tangent": (lambda: W.lq4_problem(seed=24, N=256, H=300, dt=0.005, eps=0.01),
                           dict(search=4)),
    "lq4_fp64": (lambda: W.lq4_problem(seed=24, N=200, H=300, dt=0.005, eps=0.01),
                 dict(precision=1)),
    "lq4_chance": (lambda: W.lq4_problem(seed=24, N=300, H=400, dt=0.005, eps=0.01, w_half=0.4),
                   dict(chance_q=3)),
    "fc9_grid": (lambda: W.fc9_problem(N=256, H=300, dt=0.002, w_half=0.05),
                 dict(search=1, M=16, refine=3)),
    "fc9_bisect_fp64": (lambda: W.fc9_problem(N=64, H=200, dt=0.002, w_half=0.05),
                        dict(precision=1)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_async_steps_equal_blocking_steps(R, case):
    import torch
    make, kw = CASES[case]
    p = make()
    a = R.Governor(p, **kw)
    b = R.Governor(p, **kw)
    s = torch.cuda.current_stream()
    b.set_stream(s)
    lo, hi = (-1.5, 1.5) if p.n == 4 else (0.3, 2.0)
    r_seq = W.reference_sequence(7, 6, switch_every=2, lo=lo, hi=hi)
    xs = _states(R, p, a, r_seq)
    d = _dev(torch)
    x_d = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    v_prev = float(r_seq[0]) * 0.5
    for i, r in enumerate(r_seq):
        ref = a.step(xs[i], float(r), v_prev)
        x_d.copy_(torch.from_numpy(xs[i]))
        d["r"].fill_(float(r))
        d["vp"].fill_(v_prev)
        b.step_async(x_d, d["r"], d["vp"], d["t"], d["v"], d["k"], d["st"])
        torch.cuda.synchronize()
        assert d["k"].item() == ref["kappa"], (case, i, d["k"].item(), ref["kappa"])
        assert d["v"].item() == ref["v"], (case, i)
        assert d["st"].item() == ref["status"], (case, i)
        assert d["t"].item() == i + 1
        v_prev = ref["v"]
    assert b.get_step() == 0  # the handle's own counter is untouched
    assert a.get_step() == len(r_seq)
    a.close()
    b.close()


def test_async_step_counter_selects_the_draws(R):
    # a step at device counter t equals rg_step after rg_set_step(t)
    import torch
    p = W.lq4_problem(seed=24, N=400, H=400, dt=0.005, eps=0.01, w_half=0.3)
    a = R.Governor(p)
    b = R.Governor(p)
    b.set_stream(torch.cuda.current_stream())
    d = _dev(torch)
    x = np.array([0.05, -0.1, 0.02, 0.1])
    x_d = torch.from_numpy(x).cuda()
    for t in (5, 1234, 2**31 + 17):
        a.set_step(t)
        ref = a.step(x, 1.2, 0.4)
        d["t"].fill_(t - 2**32 if t >= 2**31 else t)  # the uint32 counter in an int32 tensor
        d["r"].fill_(1.2)
        d["vp"].fill_(0.4)
        b.step_async(x_d, d["r"], d["vp"], d["t"], d["v"], d["k"], None)
        torch.cuda.synchronize()
        assert d["k"].item() == ref["kappa"] and d["v"].item() == ref["v"], t
        assert d["t"].item() & 0xFFFFFFFF == t + 1
    a.close()
    b.close()


@pytest.mark.parametrize("case", ["lq4_bisect", "fc9_grid"])
def test_captured_async_step_replays(R, case):
    import torch
    make, kw = CASES[case]
    p = make()
    a = R.Governor(p, **kw)
    g = R.Governor(p, **kw)
    cap = torch.cuda.Stream()
    g.set_stream(cap)
    d = _dev(torch)
    x_d = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    lo, hi = (-1.5, 1.5) if p.n == 4 else (0.3, 2.0)
    r_seq = W.reference_sequence(9, 5, switch_every=2, lo=lo, hi=hi)
    xs = _states(R, p, a, r_seq)
    # one eager step sets the workspace up (no allocation may happen under
    # capture); then the counter goes back to step 0
    x_d.copy_(torch.from_numpy(xs[0]))
    d["r"].fill_(float(r_seq[0]))
    torch.cuda.synchronize()
    with torch.cuda.stream(cap):
        g.step_async(x_d, d["r"], d["vp"], d["t"], d["v"], d["k"], d["st"])
    cap.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=cap):
        g.step_async(x_d, d["r"], d["vp"], d["t"], d["v"], d["k"], d["st"])
    d["t"].zero_()
    v_prev = 0.0
    for i, r in enumerate(r_seq):
        x_d.copy_(torch.from_numpy(xs[i]))
        d["r"].fill_(float(r))
        d["vp"].fill_(v_prev)
        graph.replay()
        torch.cuda.synchronize()
        ref = a.step(xs[i], float(r), v_prev)
        assert d["k"].item() == ref["kappa"], (case, i, d["k"].item(), ref["kappa"])
        assert d["v"].item() == ref["v"] and d["st"].item() == ref["status"], (case, i)
        assert d["t"].item() == i + 1
        v_prev = ref["v"]
    del graph
    g.close()
    a.close()

"""Batched serving (rg_batch_*): every instance of a mixed LQ4/FC9 batch with
uneven N and H must reach the kappa a single governor and the FP64 oracle reach."""
import numpy as np
import pytest

from paper_2510_08288_amd import workloads as W

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="batched device step switched off (rg_batch_step returns "
                            "RG_E_NOTSUP): its first device run faulted and no cause is "
                            "identified yet; the host emulation of the same kernels agrees "
                            "with the oracle"),
]


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available()
    from paper_2510_08288_amd import rg
    rg.load_library()
    return rg


def _mixed(oracle_mod, count=10, seed=3):
    rng = np.random.default_rng(seed)
    probs, xs, rs, vps = [], [], [], []
    for i in range(count):
        N = int(rng.integers(40, 600))
        H = int(rng.integers(30, 400))
        if i % 2 == 0:
            p = W.lq4_problem(seed=24 + i, N=N, H=H, dt=0.005, eps=0.01, scen_seed=100 + i,
                              instance=i)
            xs.append(np.zeros(4))
            rs.append(float(rng.uniform(-2, 2)))
            vps.append(0.0)
        else:
            p = W.fc9_problem(N=N, H=H, dt=0.002, scen_seed=200 + i, instance=i)
            xs.append(oracle_mod.Oracle(p).steady_margin(0.5)[1])
            rs.append(float(rng.uniform(1.0, 2.0)))
            vps.append(0.5)
        probs.append(p)
    return probs, xs, rs, vps


@pytest.mark.parametrize("block", [0, 64])
def test_batch_matches_single_governors_and_oracle(R, oracle_mod, block):
    probs, xs, rs, vps = _mixed(oracle_mod)
    b = R.Batch(probs, block=block, persistent_wgs=37)
    for t in range(2):  # two RG steps: fresh draws each (t advances per instance)
        out = b.step(xs, rs, vps, use_graph=(t == 1))
        for i, p in enumerate(probs):
            g = R.Governor(p, lanes=1)
            g.set_step(t)
            single = g.step(xs[i], rs[i], vps[i])
            g.close()
            ref = oracle_mod.Oracle(p, nthreads=8).bisect(xs[i], rs[i], vps[i], t, 12)
            assert out["kappa"][i] == single["kappa"], (i, t)
            assert abs(out["kappa"][i] - ref["kappa"]) <= 2.0 ** -12, (i, t)
            assert out["t"][i] == t
    b.close()


def test_batch_graph_equals_eager(R, oracle_mod):
    probs, xs, rs, vps = _mixed(oracle_mod, count=6, seed=9)
    a = R.Batch(probs)
    e = a.step(xs, rs, vps, use_graph=False)
    c = R.Batch(probs)
    g = c.step(xs, rs, vps, use_graph=True)
    assert np.array_equal(e["kappa"], g["kappa"]) and np.array_equal(e["v"], g["v"])
    a.close()
    c.close()

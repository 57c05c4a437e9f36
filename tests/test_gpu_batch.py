"""Batched serving (rg_batch_*): every instance of a mixed LQ4/FC9 batch with
uneven N and H must reach the kappa a single governor and the FP64 oracle reach."""
import numpy as np
import pytest

from paper_2510_08288_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def test_batch_mixed_generator_matches_oracle(R, oracle_mod):
    # the batched-serving generator (half 4-state, half 9-state instances, own
    # seeds, states and references) at a size the oracle checks in seconds
    insts = W.batch_instances(count=24, seed=5, n_min=64, n_max=600, h_min=50, h_max=400)
    probs = [b.problem for b in insts]
    x_fc9 = oracle_mod.Oracle(probs[1]).steady_margin(insts[1].v_prev)[1]
    xs = [b.x0 if b.x0 is not None else x_fc9 for b in insts]
    rs = [b.r for b in insts]
    vps = [b.v_prev for b in insts]
    bt = R.Batch(probs)
    outs = [bt.step(xs, rs, vps, use_graph=True) for _ in range(2)]
    bt.close()
    for t, out in enumerate(outs):
        for i, p in enumerate(probs):
            ref = oracle_mod.Oracle(p, nthreads=8).bisect(xs[i], rs[i], vps[i], t, 12)
            assert out["kappa"][i] == ref["kappa"], (t, i, out["kappa"][i], ref["kappa"])
            assert out["status"][i] == ref["status"]
    # the search runs in both plant kinds: some instances settle strictly inside (0, 1)
    kap = np.concatenate([o["kappa"] for o in outs])
    assert np.any((kap > 0) & (kap < 1)) and np.any(kap[1::2] > 0)


@pytest.mark.parametrize("depth,predict,block", [(1, False, 64), (2, True, 128), (3, False, 256)])
def test_batch_schedules_keep_kappa(R, oracle_mod, depth, predict, block):
    # search depth, first-round prediction and the scenario tile change only
    # which candidates run when: every instance's kappa is that of the default
    probs, xs, rs, vps = _mixed(oracle_mod, count=8, seed=21)
    ref = R.Batch(probs)
    a = [ref.step(xs, rs, vps, use_graph=True)["kappa"] for _ in range(2)]
    ref.close()
    b = R.Batch(probs, depth=depth, predict=predict, block=block)
    assert b.options.depth == depth and b.options.predict == int(predict)
    c = [b.step(xs, rs, vps, use_graph=True)["kappa"] for _ in range(2)]
    b.close()
    assert all(np.array_equal(x, y) for x, y in zip(a, c))


def test_batch_grid_search_matches_single_governors(R, oracle_mod):
    probs, xs, rs, vps = _mixed(oracle_mod, count=6, seed=13)
    b = R.Batch(probs, search=R.SEARCH_GRID, M=17, refine=3)
    out = b.step(xs, rs, vps, use_graph=False)
    b.close()
    for i, p in enumerate(probs):
        ref = oracle_mod.Oracle(p, nthreads=8).grid(xs[i], rs[i], vps[i], 0, 17, 3)
        assert out["kappa"][i] == ref["kappa"], (i, out["kappa"][i], ref["kappa"])


def test_batch_autotune_keeps_kappa(R, oracle_mod):
    # every schedule the batch autotuner times (tile, depth, prediction) gives
    # the same kappa; the batch created with the chosen one reproduces the
    # default batch's steps
    probs, xs, rs, vps = _mixed(oracle_mod, count=6, seed=13)
    best = R.batch_autotune(probs, xs, rs, vps)
    assert best["block"] in (64, 128, 256) and best["depth"] in (1, 2, 3)
    assert best["ms_per_batched_step"] > 0
    a = R.Batch(probs)
    ka = [a.step(xs, rs, vps, use_graph=True)["kappa"] for _ in range(3)]
    a.close()
    b = R.Batch(probs, block=best["block"], depth=best["depth"], predict=best["predict"])
    assert (b.options.block, b.options.depth) == (best["block"], best["depth"])
    kb = [b.step(xs, rs, vps, use_graph=True)["kappa"] for _ in range(3)]
    b.close()
    assert all(np.array_equal(x, y) for x, y in zip(ka, kb))

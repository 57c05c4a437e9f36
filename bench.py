#!/usr/bin/env python3
"""Closed-loop throughput of the robust reference governor on one MI355X.

Workload (synthetic, seeded): the 4-state linear-plus-quadratic closed loop,
N = 4096 disturbance scenarios, horizon H = 2000 RK4 steps of dt = 0.005, FP32
rollouts with FP64 re-simulation of lanes within 1e-4 of the constraint
boundary, 12 bisection halvings after the kappa = 1 probe, tracking a
piecewise-constant reference (levels U[-2, 2], new level every 25 steps) over
200 RG updates.

One bench step = the whole 200-update closed loop from its initial state with a
cleared search state (rg_reset): draws, every search round, rechecks,
decisions and true-plant steps, all on the device, replayed from captured HIP
graphs of generic search rounds.  Prints one JSON line.

  value       nominal scenario-steps/s: sum over the timed updates of
              (candidate evaluations sequential Alg. 1 makes) x N x H, over the
              wall time of the timed region
  roofline    the FP32 rollout kernel: executed lane RK4 steps x 356 FLOP over
              its HIP-event time (one eager loop), against the FP32 vector peak
  cpu_baseline  the FP64 oracle on this host's cores (all threads, and one
              thread), on the first RG updates of the same closed loop
  search_modes  the same closed loop under FP32 rollouts + adjoint-driven
              Newton and under plain sequential FP64 bisection, each timed in
              a child process of its own (so a kernel profile of this process
              covers the headline form only)
  extras      the other workloads, timed in a child process: one FP64 update of
              the 64-scenario plant, the 9-state adjoint workload under Newton
              and bisection, and the 9-state grid workload
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "scenario-steps/s + RG updates/s at κ tol 2^-12 (FP32+adjoint vs FP64 bisect)"
# Algorithmic FLOP of one LQ4 scenario-step (FMA = 2): 4 stages x 68 (x.*x and the
# 4 x 8 [A G] product) + 24 (stage inputs) + 24 (update) + 16 (E w) + 20 (C x,
# margin rows, minimum).
FLOP_PER_STEP_LQ4 = 356
FLOP_PER_STEP_FC9 = 1055     # same for FC9, plus 36 tanh, 24 sqrt and 1 division
BYTES_PER_STEP_LQ4 = 8       # streamed draws read per scenario-step (2 x fp32)
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak (needs packed FP32)
PEAK_FP32_NONPACKED_TFLOPS = 78.6
# HBM bytes per rollout launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of
# this bench, each scaled by the counter's reading for a device copy of known size;
# valid only for the kernel sources they were taken on (SHA-1 of the device sources
# below, concatenated in this order).
KERNEL_SOURCES = ("rg_kernels.hip", "rg_device.hpp", "rg_internal.hpp")
HBM_TRAFFIC = {"kernels_sha1": "c1d43d815060d5efe28c0b2f2e2ddf994d19b6f6", "bytes_per_launch": 110040372}
FIXTURE = os.path.join(ROOT, "tests", "golden", "lq4_closed_loop_n4096_h2000.txt")


def cpu_baseline(wl, seconds, single_seconds):
    """The FP64 oracle, as it stands, on the host's cores: RG updates of the same
    closed loop from its start until `seconds` have elapsed (all threads), then
    the same with one thread for `single_seconds`."""
    import numpy as np

    from oracle import oracle as O

    p = wl["problem"]
    r_seq = wl["r_seq"]

    def run(threads, budget):
        o = O.Oracle(p, nthreads=threads)
        x = np.asarray(wl["x0"], dtype=np.float64)
        v_prev = wl["v_prev"]
        steps = nominal = 0
        kappas = []
        t0 = time.perf_counter()
        while True:
            res = o.bisect(x, r_seq[steps], v_prev, steps, wl["K"])
            kappas.append(res["kappa"])
            nominal += res["passes"] * p.N * p.H
            x = o.plant_step(x, res["v"], steps)
            v_prev = res["v"]
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget or steps >= len(r_seq):
                return nominal / el, steps / el, steps, el, kappas

    threads = os.cpu_count() or 1
    val, ups, steps, el, kappas = run(threads, seconds)
    val1, ups1, steps1, el1, _ = run(1, single_seconds)
    return dict(value=val, unit="scenario-steps/s", cores=threads, kind="oracle",
                rg_updates_per_s=ups,
                sample=f"first {steps} RG updates of the same closed loop (N={p.N}, H={p.H}), "
                       f"FP64 bisection, {threads} threads over scenarios, {el:.1f} s",
                single_thread={"value": val1, "rg_updates_per_s": ups1, "cores": 1,
                               "sample": f"first {steps1} RG updates, 1 thread, {el1:.1f} s"}), kappas


def measured_traffic():
    """roofline.traffic: the counter-based HBM bytes per rollout launch, or None
    once the kernel source differs from the one the counters were taken on."""
    import hashlib
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_08288_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    sha = h.hexdigest()
    return HBM_TRAFFIC["bytes_per_launch"] if sha == HBM_TRAFFIC["kernels_sha1"] else None


def fixture_kappa():
    """kappa of every update of the FP64 oracle's closed loop (tests/golden), or None."""
    if not os.path.exists(FIXTURE):
        return None
    rows = [ln.split() for ln in open(FIXTURE) if ln.strip() and not ln.startswith("#")]
    return [float(r[7]) for r in rows]


def _loop(g, x0, v0, r_seq, use_graph):
    """One full closed loop from the initial state with a cleared search state."""
    g.reset()
    g.set_step(0)
    return g.closed_loop(x0, v0, r_seq, use_graph=use_graph)


def run_form(args):
    """One alternative search form over the whole closed loop, replayed from
    captured HIP graphs; then the headline form (FP32 bisection) at every state
    of this form's own loop.  Prints one JSON line."""
    import numpy as np
    import torch

    from paper_2510_08288_amd import rg, workloads as W

    wl = W.workload_lq4_closed_loop(T=200)
    p = wl["problem"]
    r_seq = wl["r_seq"]
    T = len(r_seq)
    kw = {"fp32_adjoint_newton": dict(precision=rg.PREC_F32_RECHECK, search=rg.SEARCH_NEWTON),
          "fp32_tangent_newton": dict(precision=rg.PREC_F32_RECHECK, search=rg.SEARCH_NEWTON_TAN),
          "fp64_sequential_bisection": dict(precision=rg.PREC_F64, depth=1, predict=False)}[args.form]
    gm = rg.Governor(p, band=wl["band"], K=wl["K"], max_T=256, **kw)
    x0 = np.asarray(wl["x0"], dtype=np.float64)
    _loop(gm, x0, wl["v_prev"], r_seq, True)  # captures the graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    om = _loop(gm, x0, wl["v_prev"], r_seq, True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gm.close()
    gb = rg.Governor(p, band=wl["band"], K=wl["K"])
    kb = np.zeros(T)
    for s in range(T):
        gb.set_step(s)
        kb[s] = gb.step(om["x"][s], r_seq[s], wl["v_prev"] if s == 0 else om["v"][s - 1])["kappa"]
    gb.close()
    d = np.abs(om["kappa"] - kb)
    print(json.dumps({"rg_updates_per_s": T / el, "ms_per_update": el / T * 1e3, "updates": T,
                      "value": float(np.sum(om["bisect_passes"])) * p.N * p.H / el,
                      "rounds_per_update": float(np.mean(om["rounds"])),
                      "fallback_updates": int(np.sum(om["status"] == 2)),
                      "max_abs_kappa_diff_vs_bisection_same_state": float(np.max(d)),
                      "kappa_within_2^-12": bool(np.all(d <= 2.0 ** -wl["K"] + 1e-15)),
                      "kappa": [float(k) for k in om["kappa"]]}))


def run_extras(args):
    """The other named workloads, in a child process: prints one JSON line."""
    import numpy as np
    import torch

    from paper_2510_08288_amd import rg, workloads as W

    out = {}
    # one FP64 update of the 64-scenario LQ4 plant (plain FP64 scenario RG)
    w1 = W.workload_lq4_fp64_single()
    g = rg.Governor(w1["problem"], precision=rg.PREC_F64, K=w1["K"])
    times = []
    for rep in range(21):
        g.set_step(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = g.step(w1["x0"], w1["r"], w1["v_prev"])
        times.append(time.perf_counter() - t0)
    g.close()
    p1 = w1["problem"]
    ms = float(np.median(times[1:])) * 1e3
    out["lq4_fp64_n64_h500"] = {"ms_per_update": ms, "rg_updates_per_s": 1e3 / ms,
                                "value": res["bisect_passes"] * p1.N * p1.H / (ms * 1e-3),
                                "kappa": res["kappa"], "passes": res["bisect_passes"],
                                "unit": "scenario-steps/s", "precision": "fp64",
                                "timing": "median of 20 blocking rg_step calls"}
    # the 9-state adjoint workload: FP32 + adjoint-driven Newton against plain
    # sequential FP64 bisection and FP32 speculative bisection, updates at t = 0..U-1
    wa = W.workload_fc9_adjoint()
    pa = wa["problem"]
    U = args.extra_updates
    forms = {"fp32_adjoint_newton": dict(precision=rg.PREC_F32_RECHECK, search=rg.SEARCH_NEWTON,
                                         Kc=wa["Kc"]),
             "fp32_tangent_newton": dict(precision=rg.PREC_F32_RECHECK,
                                         search=rg.SEARCH_NEWTON_TAN),
             "fp64_sequential_bisection": dict(precision=rg.PREC_F64, depth=1, predict=False),
             "fp32_speculative_bisection": dict(precision=rg.PREC_F32_RECHECK)}
    c4 = {"workload": wa["name"], "updates": U}
    kap = {}
    x0 = None
    for name, kw in forms.items():
        g = rg.Governor(pa, K=wa["K"], **kw)
        if x0 is None:
            x0 = g.equilibrium(wa["v_prev"])
        g.set_step(0)
        g.step(x0, wa["r"], wa["v_prev"])  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = []
        for t in range(U):
            g.set_step(t)
            res.append(g.step(x0, wa["r"], wa["v_prev"]))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g.close()
        kap[name] = np.array([r["kappa"] for r in res])
        c4[name] = {"ms_per_update": el / U * 1e3, "rg_updates_per_s": U / el,
                    "value": sum(r["bisect_passes"] for r in res) * pa.N * pa.H / el,
                    "rounds_per_update": float(np.mean([r["rounds"] for r in res])),
                    "kappa": [float(k) for k in kap[name]]}
    for nm in ["fp32_adjoint_newton", "fp32_tangent_newton"]:
        dn = np.abs(kap[nm] - kap["fp64_sequential_bisection"])
        c4[nm]["max_abs_kappa_diff_vs_fp64_bisection"] = float(np.max(dn))
        c4[nm]["kappa_within_2^-12"] = bool(np.all(dn <= 2.0 ** -wa["K"] + 1e-15))
        c4[nm]["speedup_vs_fp64_bisection"] = (c4["fp64_sequential_bisection"]["ms_per_update"] /
                                               c4[nm]["ms_per_update"])
    out["fc9_adjoint_n16384_h1000"] = c4
    out.update(run_fc9_grid(U, rg, W, np, torch))
    out.update(run_more_extras(rg, W, np, torch))
    print(json.dumps(out))


def run_fc9_grid(U, rg, W, np, torch):
    """The 9-state grid workload (N = 65536, H = 1000, 64-point grid + 6
    refinements): U updates at t = 0..U-1 after one warm-up, rollout launches
    timed with HIP events."""
    out = {}
    wg = W.workload_fc9_grid()
    pg = wg["problem"]
    g = rg.Governor(pg, search=rg.SEARCH_GRID, M=wg["M"], refine=wg["refine"], band=wg["band"])
    xg = g.equilibrium(wg["v_prev"])
    g.set_step(0)
    g.step(xg, wg["r"], wg["v_prev"])  # warm-up
    g.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for t in range(U):
        g.set_step(t)
        res.append(g.step(xg, wg["r"], wg["v_prev"]))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = g.profile()
    g.close()
    out[wg["name"]] = {
        "updates": U, "ms_per_update": el / U * 1e3, "kappa": [r["kappa"] for r in res],
        "rounds_per_update": float(np.mean([r["rounds"] for r in res])),
        "rechecks_per_update": float(np.mean([r["rechecks"] for r in res])),
        "value": sum(r["bisect_passes"] for r in res) * pg.N * pg.H / el,
        "executed_scenario_steps_per_s": sum(r["lane_steps"] for r in res) / el,
        "rollout_ms_per_update": prof["rollout_ms"] / U,
        "rollout_tflops": (prof["lane_steps"] * FLOP_PER_STEP_FC9 / (prof["rollout_ms"] * 1e-3) / 1e12
                           if prof["rollout_ms"] > 0 else 0.0),
        "flop_per_scenario_step": FLOP_PER_STEP_FC9, "unit": "scenario-steps/s"}
    return out


def _median_ms(fn, reps):
    import torch
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t0)
    return float(sorted(times)[len(times) // 2]) * 1e3


def run_more_extras(rg, W, np, torch):
    """Alg. 2 (per-scenario bisection), the chance-constrained verdict and the
    allocation-free step, each timed on the workloads above."""
    out = {}
    # Alg. 2 on the 64-scenario FP64 update and on one update of the 4-state
    # bench workload (a state where the search runs: kappa strictly inside)
    w1 = W.workload_lq4_fp64_single()
    wl = W.workload_lq4_closed_loop(T=40)
    xs = np.array([0.12, -0.05, 0.3, -0.2])
    alg2 = {}
    for name, prob, prec, x, r, vp, t in [
            ("lq4_fp64_n64_h500", w1["problem"], rg.PREC_F64, w1["x0"], w1["r"], w1["v_prev"], 0),
            ("lq4_n4096_h2000_one_update", wl["problem"], rg.PREC_F32_RECHECK, xs, 1.9, 0.4, 26)]:
        res = {}
        for form, kw in [("alg2", dict(search=rg.SEARCH_ALG2)), ("bisection", dict())]:
            g = rg.Governor(prob, precision=prec, K=12, **kw)
            last = {}

            def one():
                g.set_step(t)
                last.update(g.step(x, r, vp))
            ms = _median_ms(one, 9)
            g.close()
            res[form] = {"ms_per_update": ms, "kappa": last["kappa"],
                         "passes": last["bisect_passes"]}
        res["same_kappa"] = res["alg2"]["kappa"] == res["bisection"]["kappa"]
        alg2[name] = res
    out["alg2_per_scenario_bisection"] = alg2
    # chance-constrained verdict (at most q of N scenarios may violate) on the
    # 4-state bench closed loop, first 50 updates, graph replay
    wc = W.workload_lq4_closed_loop(T=50)
    cc = {}
    for q in (0, 4, 41):
        g = rg.Governor(wc["problem"], band=wc["band"], K=wc["K"], chance_q=q, max_T=256)
        g.closed_loop(wc["x0"], wc["v_prev"], wc["r_seq"], use_graph=True)  # capture
        g.reset()
        g.set_step(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = g.closed_loop(wc["x0"], wc["v_prev"], wc["r_seq"], use_graph=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g.close()
        cc[f"q={q}"] = {"ms_per_update": el / len(wc["r_seq"]) * 1e3,
                        "mean_kappa": float(np.mean(o["kappa"])),
                        "infeasible_updates": int(np.sum(o["status"] != 0))}
    cc["updates"] = len(wc["r_seq"])
    cc["N"] = wc["problem"].N
    out["chance_constrained_lq4_closed_loop"] = cc
    # allocation-free step against rg_step on one update of the bench workload
    ga = rg.Governor(wl["problem"], band=wl["band"], K=wl["K"], torch_workspace=False)
    gb = rg.Governor(wl["problem"], band=wl["band"], K=wl["K"])
    ra, rb = {}, {}

    def na():
        ga.set_step(26)
        ra.update(ga.step_noalloc(xs, 1.9, 0.4))

    def st():
        gb.set_step(26)
        gb.reset()
        rb.update(gb.step(xs, 1.9, 0.4))
    out["noalloc_step_lq4_n4096_h2000"] = {"noalloc_ms": _median_ms(na, 9),
                                           "rg_step_ms": _median_ms(st, 9),
                                           "same_kappa": ra["kappa"] == rb["kappa"]}
    ga.close()
    gb.close()
    # the step on device pointers, captured once as a CUDA graph and replayed,
    # against rg_step on the same update (both repeat the update without
    # clearing the search record in between)
    gc = rg.Governor(wl["problem"], band=wl["band"], K=wl["K"])
    gd = rg.Governor(wl["problem"], band=wl["band"], K=wl["K"])
    cap = torch.cuda.Stream()
    gc.set_stream(cap)
    f64 = dict(dtype=torch.float64, device="cuda")
    x_d = torch.from_numpy(np.asarray(xs, dtype=np.float64)).cuda()
    r_d, vp_d = torch.full((1,), 1.9, **f64), torch.full((1,), 0.4, **f64)
    v_d, k_d = torch.zeros(1, **f64), torch.zeros(1, **f64)
    t_d = torch.full((1,), 26, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(cap):
        gc.step_async(x_d, r_d, vp_d, t_d, v_d, k_d)  # sets the workspace up
    cap.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=cap):
        gc.step_async(x_d, r_d, vp_d, t_d, v_d, k_d)
    rd = {}

    def replay():
        t_d.fill_(26)
        graph.replay()
        torch.cuda.synchronize()

    def blocking():
        gd.set_step(26)
        rd.update(gd.step(xs, 1.9, 0.4))
    out["async_step_graph_lq4_n4096_h2000"] = {"graph_replay_ms": _median_ms(replay, 9),
                                               "rg_step_ms": _median_ms(blocking, 9),
                                               "same_kappa": k_d.item() == rd["kappa"]}
    del graph
    gc.close()
    gd.close()
    out["batch_1024_lq4_fc9"] = run_batch(rg, W, np, torch)
    # points of the paper-shaped sweep (bench.py --paper-sweep runs all 288)
    ns = [1, 32, 256, 512, 1024, 1312, 2048, 4096, 8192]
    out["paper_sweep_fc9_grid_m32_h1024"] = {
        "rows": paper_sweep_rows(ns, [("streamed_ms", rg.RNG_STREAM)], log_every=1 << 30),
        "timing": "median of five blocking rg_step calls after one warm-up, fresh handle per N"}
    return out


def run_batch(rg, W, np, torch, steps=2):
    """Batched serving: 1024 independent instances (512 four-state, 512
    nine-state), N ~ U{256..8192}, H ~ U{200..3000}, dt = 0.005, own seeds,
    states and references; every batched RG step replayed from one captured
    graph.  The first step captures the graph and is not timed."""
    insts = W.batch_instances(count=1024)
    probs = [b.problem for b in insts]
    # the 9-state instances start at the nominal equilibrium of their v_prev
    # (shared plant): one device equilibrium serves them all
    ge = rg.Governor(probs[1])
    x_fc9 = ge.equilibrium(insts[1].v_prev)
    ge.close()
    xs = [b.x0 if b.x0 is not None else x_fc9 for b in insts]
    rs = [b.r for b in insts]
    vps = [b.v_prev for b in insts]
    t0 = time.perf_counter()
    bt = rg.Batch(probs)
    bt.step(xs, rs, vps, use_graph=True)  # allocates, captures, runs step 0
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    outs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        outs.append(bt.step(xs, rs, vps, use_graph=True))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    depth = bt.options.depth
    bt.close()
    # the batch autotuner on the whole batch (18 schedules, three steps each),
    # then the batch under the schedule it chose
    t2 = time.perf_counter()
    best = rg.batch_autotune(probs, xs, rs, vps)
    tune_s = time.perf_counter() - t2
    bt = rg.Batch(probs, block=best["block"], depth=best["depth"], predict=best["predict"])
    bt.step(xs, rs, vps, use_graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tuned = [bt.step(xs, rs, vps, use_graph=True) for _ in range(steps)]
    torch.cuda.synchronize()
    el_tuned = time.perf_counter() - t1
    bt.close()
    tuned_same = all(np.array_equal(a["kappa"], b["kappa"]) for a, b in zip(outs, tuned))
    NH = np.array([p.N * p.H for p in probs], dtype=np.float64)
    nominal = sum(float(np.sum(o["bisect_passes"] * NH)) for o in outs)
    executed = sum(float(np.sum(o["lane_steps"])) for o in outs)
    return {"instances": len(probs), "steps_timed": steps,
            "ms_per_batched_step": el / steps * 1e3,
            "instance_updates_per_s": len(probs) * steps / el,
            "value": nominal / el, "unit": "scenario-steps/s",
            "executed_scenario_steps_per_s": executed / el,
            "mean_rounds": float(np.mean([np.mean(o["rounds"]) for o in outs])),
            "infeasible_instance_updates": int(sum(np.sum(o["status"] != 0) for o in outs)),
            "mean_kappa_lq4": float(np.mean([np.mean(o["kappa"][0::2]) for o in outs])),
            "mean_kappa_fc9": float(np.mean([np.mean(o["kappa"][1::2]) for o in outs])),
            "first_step_with_capture_s": first,
            "sum_N_x_H": float(np.sum(NH)), "depth_instance0": int(depth),
            "autotuned": {"schedule": {k: best[k] for k in ("block", "depth", "predict")},
                          "tuner_ms_per_batched_step": best["ms_per_batched_step"],
                          "ms_per_batched_step": el_tuned / steps * 1e3,
                          "same_kappa_as_default": bool(tuned_same),
                          "tuning_s": tune_s}}


def paper_sweep_rows(Ns, modes, reps=6, log_every=1024):
    """RG-step time of the 9-state grid search (Alg. 3, M = 32 points, no
    refinement), H = 1024, dt = 0.01, from the nominal equilibrium of v = 0.5
    towards r = 2.0, for each N in Ns: a fresh handle per N and draw mode, the
    median of reps - 1 blocking steps after one warm-up.  With streamed draws
    the row also gives `rollout_ms`, the mean time per step of the rollout
    launches alone (HIP events around them; no draw generation, transfers,
    recheck or decision), the counterpart of the paper's second GPU timing,
    which leaves out scenario generation and transfers."""
    import numpy as np
    import torch

    from paper_2510_08288_amd import rg, workloads as W

    rows = []
    x0 = None
    for N in Ns:
        p = W.fc9_problem(N=N, H=1024, dt=0.01)
        row = {"N": N}
        for label, mode in modes:
            g = rg.Governor(p, search=rg.SEARCH_GRID, M=32, refine=0, rng_mode=mode)
            if x0 is None:
                x0 = g.equilibrium(0.5)
            times = []
            for rep in range(reps):
                g.set_step(0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = g.step(x0, 2.0, 0.5)
                times.append(time.perf_counter() - t0)
            row["lanes"] = int(g.options.lanes)
            if mode == rg.RNG_STREAM:
                g.set_profiling(True)
                for rep in range(reps - 1):
                    g.set_step(0)
                    g.step(x0, 2.0, 0.5)
                pf = g.profile()
                row["rollout_ms"] = pf["rollout_ms"] / (reps - 1)
                g.set_profiling(False)
            g.close()
            row[label] = float(np.median(times[1:])) * 1e3
            row["kappa"] = res["kappa"]
            row["rechecks"] = res["rechecks"]
        # every N has workspaces of its own size: hand them back to the device
        torch.cuda.empty_cache()
        rows.append(row)
        if N % log_every == 0 or N == 32:
            progress(f"paper sweep N={N}: {row}")
    return rows


def run_paper_sweep(args):
    """Shape of the paper's GPU timing experiment (Sec. IV-B): the 9-state plant
    with the grid search of Alg. 3 (M = 32 points, no refinement), H = 1024,
    dt = 0.01, N = 1..32 and 32..8192 in steps of 32 (or the --sweep-n list);
    per N the median of five blocking RG steps with the draws generated into
    device memory first (streamed) and with the draws generated inside the
    rollout lanes (inline).  Prints one JSON line."""
    from paper_2510_08288_amd import rg

    Ns = ([int(n) for n in args.sweep_n.split(",")] if args.sweep_n
          else list(range(1, 33)) + list(range(64, 8193, 32)))
    rows = paper_sweep_rows(Ns, [("streamed_ms", rg.RNG_STREAM), ("inline_ms", rg.RNG_INLINE)])
    print(json.dumps({"workload": "fc9_grid_m32_h1024_dt0.01", "rows": rows}))


def progress(msg):
    """One progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def child(args, *extra):
    proc = subprocess.run([sys.executable, os.path.abspath(__file__), *extra], capture_output=True,
                          text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise SystemExit(f"{' '.join(extra)} failed (exit {proc.returncode})")
    return json.loads(proc.stdout.strip().splitlines()[-1])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed closed loops (200 updates each)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed closed loops before them")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-single-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--depth", type=int, default=0)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--block", type=int, default=0, help="rollout workgroup (0: library choice)")
    ap.add_argument("--speculate", type=int, default=-1,
                    help="speculation depth with --no-autotune (-1: library default)")
    ap.add_argument("--form", choices=["fp32_adjoint_newton", "fp32_tangent_newton",
                                       "fp64_sequential_bisection"],
                    default=None, help=argparse.SUPPRESS)
    ap.add_argument("--extras-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--paper-sweep", action="store_true",
                    help="only the paper-shaped sweep of RG-step time against N (9-state grid, "
                         "M = 32) and exit")
    ap.add_argument("--sweep-n", default="", help="comma-separated N list for --paper-sweep")
    ap.add_argument("--extra-updates", type=int, default=3,
                    help="updates timed per form on the 9-state workloads")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads and the alternative search forms")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default schedule instead of the autotuned one")
    ap.add_argument("--tune-steps", type=int, default=200,
                    help="closed-loop updates the autotuner times each schedule on")
    ap.add_argument("--autotune-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--fc9-grid-only", action="store_true",
                    help="only the 9-state grid workload (--extra-updates updates) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy one device buffer of BYTES into another three times (the "
                         "reference kernel for scaling HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the scenario axis would "
              "shard over GPUs with one min-reduction per search round, which this build does "
              "not implement.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2510_08288_amd import rg, workloads as W

    torch.cuda.set_device(0)
    if args.form is not None:
        return run_form(args)
    if args.fc9_grid_only:
        print(json.dumps(run_fc9_grid(args.extra_updates, rg, W, np, torch)))
        return
    if args.extras_only:
        return run_extras(args)
    if args.paper_sweep:
        return run_paper_sweep(args)
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration, "copies": 3}))
        return
    wl = W.workload_lq4_closed_loop(T=200)
    p = wl["problem"]
    r_seq = wl["r_seq"]
    T = len(r_seq)
    x0 = np.asarray(wl["x0"], dtype=np.float64)
    v0 = wl["v_prev"]
    if args.autotune_only:
        ga = rg.Governor(p, band=wl["band"], K=wl["K"], max_T=256)
        ga.set_step(0)
        print(json.dumps(ga.autotune(x0, v0, r_seq[: args.tune_steps])))
        ga.close()
        return

    # launch schedule (lanes per scenario, workgroup, search depth, first-round
    # prediction, speculation) from the autotuner, timed on the workload's first
    # updates in a child process of its own (its trial launches stay out of this
    # process)
    tuned = None
    sched = dict(depth=args.depth, lanes=args.lanes, block=args.block)
    if args.speculate >= 0:
        sched["speculate"] = args.speculate
    if not args.no_autotune and args.tune_steps > 0:
        tuned = child(args, "--autotune-only", "--tune-steps", str(args.tune_steps))
        progress(f"autotuned schedule {tuned}")
        sched = dict(depth=tuned["depth"], lanes=tuned["lanes"], block=tuned["block"],
                     predict=bool(tuned["predict"]), speculate=int(tuned["speculate"]))
    g = rg.Governor(p, band=wl["band"], K=wl["K"], max_T=256, **sched)

    # warm-up loops (the first captures the graphs), untimed
    warm_launches = 0  # rollout launches before the profiled loop (one per round, >= 1 per update)
    for _ in range(max(1, args.warmup)):
        ow = _loop(g, x0, v0, r_seq, True)
        warm_launches += int(np.sum(np.maximum(1, np.asarray(ow["rounds"]))))

    # one loop launched eagerly with a HIP event pair around every rollout launch
    # (the roofline figure); untimed
    g.set_profiling(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out_e = _loop(g, x0, v0, r_seq, False)
    torch.cuda.synchronize()
    elapsed_eager = time.perf_counter() - t1
    prof = g.profile()
    g.set_profiling(False)

    # timed region: K whole closed loops replayed from the captured graphs
    outs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outs.append(_loop(g, x0, v0, r_seq, True))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    progress(f"{args.steps} timed closed loops: {elapsed:.3f} s")
    out = outs[0]
    same = all(np.array_equal(o["v"], out["v"]) and np.array_equal(o["x"], out["x"]) for o in outs)
    graph_same = bool(np.array_equal(out_e["v"], out["v"]))
    g.close()

    modes, extras = {}, {}
    if not args.no_extras:
        for label in ["fp32_adjoint_newton", "fp32_tangent_newton", "fp64_sequential_bisection"]:
            om = child(args, "--form", label)
            kap = np.asarray(om.pop("kappa"))
            om["same_closed_loop_as_headline"] = bool(np.array_equal(kap, out["kappa"]))
            modes[label] = om
            progress(f"search form {label}: {om['ms_per_update']:.3f} ms per update")
        extras = child(args, "--extras-only", "--extra-updates", str(args.extra_updates))

    K = args.steps
    updates = K * T
    passes = int(np.sum(out["bisect_passes"]))
    nominal = passes * p.N * p.H * K
    executed = int(np.sum(out["lane_steps"])) * K
    value = nominal / elapsed
    flops = prof["lane_steps"] * FLOP_PER_STEP_LQ4
    kern_s = prof["rollout_ms"] * 1e-3
    achieved = flops / kern_s / 1e12 if kern_s > 0 else 0.0
    ref_k = fixture_kappa()
    oracle_check = None
    if ref_k is not None and len(ref_k) == T:
        dk = np.abs(np.asarray(ref_k) - out["kappa"])
        oracle_check = {"updates": T, "identical": bool(np.all(dk == 0)),
                        "max_abs_kappa_diff": float(np.max(dk)),
                        "within_2^-12": bool(np.all(dk <= 2.0 ** -wl["K"]))}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "scenario-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "plant": "LQ4", "N": p.N, "H": p.H, "dt": p.dt,
                   "K": wl["K"], "band": wl["band"], "rg_updates_per_step": T,
                   "step": "one whole closed loop of 200 RG updates from the initial state, "
                           "search state cleared",
                   "precision": "fp32 rollouts + fp64 near-band recheck",
                   "search": "bisection: first device round = kappa 1 probe + the midpoints on "
                             "the path to the previous update's kappa, then "
                             f"{sched.get('depth') or 'auto'} levels per round",
                   "lanes_per_scenario": sched.get("lanes"),
                   "workgroup": sched.get("block") or 256,
                   "first_round_prediction": bool(sched.get("predict", True)),
                   "speculation_depth": int(sched.get("speculate", 7)),
                   "schedule": ("autotuned on the first %d updates" % args.tune_steps
                                if tuned else "library default or command line"),
                   "launch": "captured HIP graphs of generic search rounds, replayed until "
                             "every update is recorded"},
        "rg_updates_per_s": updates / elapsed,
        "ms_per_update": elapsed / updates * 1e3,
        "executed_scenario_steps_per_s": executed / elapsed,
        "timed_loops_identical": same,
        "kappa_vs_fp64_oracle_fixture": oracle_check,
        "eager_profiled": {"ms_per_update": elapsed_eager / T * 1e3,
                           "rg_updates_per_s": T / elapsed_eager,
                           "value": passes * p.N * p.H / elapsed_eager, "same_result": graph_same},
        "search_modes": dict(modes, fp32_speculative_bisection={
            "rg_updates_per_s": updates / elapsed, "ms_per_update": elapsed / updates * 1e3,
            "updates": T, "rounds_per_update": float(np.mean(out["rounds"]))}),
        "extras": extras,
        "search_stats": {"updates": T, "rounds": int(np.sum(out["rounds"])),
                         "candidates": int(np.sum(out["candidates"])),
                         "rechecks": int(np.sum(out["rechecks"])),
                         "bisect_passes": passes,
                         "updates_with_more_than_one_candidate":
                             int(np.sum(np.asarray(out["bisect_passes"]) > 1)),
                         "infeasible_updates": int(np.sum(out["status"] != 0))},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic() if sched.get("lanes") == 4 else None,
                     "kernel": ("k_rollout_lq4_quad (one scenario per 4 lanes)"
                                if sched.get("lanes") == 4 else "k_rollout<LQ4, float>"),
                     "launches": prof["rollout_launches"],
                     "launches_before": warm_launches,
                     "avg_launch_ms": prof["rollout_ms"] / max(1, prof["rollout_launches"]),
                     "flop_per_scenario_step": FLOP_PER_STEP_LQ4,
                     "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                     "frac_of_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                     "achieved_hbm_gbs": prof["lane_steps"] * BYTES_PER_STEP_LQ4 / kern_s / 1e9
                     if kern_s > 0 else 0.0},
    }
    progress("other workloads done")
    if not args.no_cpu_baseline:
        base, kappas = cpu_baseline(wl, args.cpu_seconds, args.cpu_single_seconds)
        n = len(kappas)
        base["kappa_equal_first_updates"] = bool(np.array_equal(np.asarray(kappas), out["kappa"][:n]))
        line["cpu_baseline"] = base
    print(json.dumps(line))


if __name__ == "__main__":
    main()

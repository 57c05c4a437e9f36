#!/usr/bin/env python3
"""Closed-loop throughput of the robust reference governor on one MI355X.

Workload (synthetic, seeded): the 4-state linear-plus-quadratic closed loop,
N = 4096 disturbance scenarios, horizon H = 2000 RK4 steps of dt = 0.005, FP32
rollouts with FP64 re-simulation of lanes within 1e-4 of the constraint
boundary, 12 bisection halvings after the kappa = 1 probe, tracking a
piecewise-constant reference (levels U[-2, 2], new level every 25 steps).

One bench step = one RG update of that closed loop (draws, all search rounds,
recheck, decision, true-plant step), all on the device, replayed from the HIP
graph captured for one RG step.  Prints one JSON line.

  value       nominal scenario-steps/s: sum over the timed RG updates of
              (candidate evaluations sequential Alg. 1 makes) x N x H, over the
              wall time of the timed region
  roofline    the FP32 rollout kernel: executed lane RK4 steps x 375 FLOP over
              its HIP-event time, against the FP32 vector peak
  cpu_baseline  the FP64 reference on this host's cores, on the first RG
              updates of the same closed loop
  search_modes  the same closed loop under FP32 rollouts + adjoint-driven
              Newton and under plain sequential FP64 bisection, each timed in
              a child process of its own (so a kernel profile of this process
              covers the headline form only)
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
FLOP_PER_STEP_LQ4 = 375      # algorithmic FLOP of one LQ4 scenario-step (FMA = 2)
FLOP_PER_STEP_FC9 = 1055     # same for FC9, plus 36 tanh, 24 sqrt and 1 division
BYTES_PER_STEP_LQ4 = 8       # streamed draws read per scenario-step (2 x fp32)
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak (needs packed FP32)
PEAK_FP32_NONPACKED_TFLOPS = 78.6
# HBM bytes per rollout launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of
# this bench (4 updates), each scaled by the counter's reading for a 256 MiB device
# copy; valid only for the kernel sources they were taken on (SHA-1 of the device
# sources below, concatenated in this order).
KERNEL_SOURCES = ("rg_kernels.hip", "rg_device.hpp", "rg_internal.hpp")
HBM_TRAFFIC = {"kernels_sha1": "7043151f7f6d91cc4173879fe1c87618cb5e05c3",
               "bytes_per_launch": 106314480}


def cpu_baseline(wl, r_seq, seconds):
    """The FP64 reference, as it stands, on the host's cores: RG updates of the
    same closed loop from its start, until `seconds` have elapsed."""
    import numpy as np

    from oracle import oracle as O

    p = wl["problem"]
    threads = os.cpu_count() or 1
    o = O.Oracle(p, nthreads=threads)
    x = np.asarray(wl["x0"], dtype=np.float64)
    v_prev = wl["v_prev"]
    steps = 0
    nominal = 0
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
        if el >= seconds or steps >= len(r_seq):
            break
    return dict(value=nominal / el, unit="scenario-steps/s", cores=threads, kind="oracle",
                rg_updates_per_s=steps / el,
                sample=f"first {steps} RG updates of the same closed loop (N={p.N}, H={p.H}), "
                       f"FP64 bisection, {threads} threads over scenarios, {el:.1f} s"), kappas


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


def fc9_grid_measurement(args, updates: int = 3):
    """Secondary measurement: RG updates of the 9-state grid workload (64-point
    grid + 6 refinements, N = 65536, H = 1000), each a separate update at its own
    draws (t = 0, 1, ...) from the equilibrium of v_prev."""
    import numpy as np
    import torch

    from paper_2510_08288_amd import rg, workloads as W

    wl = W.workload_fc9_grid()
    p = wl["problem"]
    g = rg.Governor(p, search=rg.SEARCH_GRID, M=wl["M"], refine=wl["refine"], band=wl["band"])
    x0 = g.equilibrium(wl["v_prev"])
    g.set_step(0)
    g.step(x0, wl["r"], wl["v_prev"])  # warm-up (kernel loading, draws)
    g.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for t in range(updates):
        g.set_step(t)
        res.append(g.step(x0, wl["r"], wl["v_prev"]))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = g.profile()
    g.close()
    nominal = sum(r["bisect_passes"] for r in res) * p.N * p.H
    executed = sum(r["lane_steps"] for r in res)
    return {"workload": wl["name"], "updates": updates, "ms_per_update": el / updates * 1e3,
            "kappa": [r["kappa"] for r in res], "rounds_per_update": float(np.mean([r["rounds"] for r in res])),
            "value": nominal / el, "executed_scenario_steps_per_s": executed / el,
            "rollout_ms_per_update": prof["rollout_ms"] / updates,
            "rollout_tflops": (prof["lane_steps"] * FLOP_PER_STEP_FC9 / (prof["rollout_ms"] * 1e-3) / 1e12
                               if prof["rollout_ms"] > 0 else 0.0),
            "flop_per_scenario_step": FLOP_PER_STEP_FC9,
            "unit": "scenario-steps/s"}


def run_form(args):
    """One alternative search form on the first `--steps` updates of the same
    closed loop, replayed from captured HIP graphs; prints one JSON line."""
    import numpy as np
    import torch

    from paper_2510_08288_amd import rg, workloads as W

    T = args.steps
    wl = W.workload_lq4_closed_loop(T=max(T, 2))
    p = wl["problem"]
    r_seq = wl["r_seq"]
    kw = (dict(precision=rg.PREC_F32_RECHECK, search=rg.SEARCH_NEWTON)
          if args.form == "fp32_adjoint_newton"
          else dict(precision=rg.PREC_F64, depth=1, predict=False))
    gm = rg.Governor(p, band=wl["band"], K=wl["K"], max_T=max(256, T), **kw)
    x0 = np.asarray(wl["x0"], dtype=np.float64)
    gm.set_step(0)
    gm.closed_loop(x0, wl["v_prev"], r_seq[:2], use_graph=True)  # capture + warm the graph
    gm.set_step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    om = gm.closed_loop(x0, wl["v_prev"], r_seq[:T], use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gm.close()
    print(json.dumps({"rg_updates_per_s": T / el, "ms_per_step": el / T * 1e3, "steps": T,
                      "value": float(np.sum(om["bisect_passes"])) * p.N * p.H / el,
                      "rounds_per_step": float(np.mean(om["rounds"])),
                      "fallback_steps": int(np.sum(om["status"] == 2)),
                      "kappa": [float(k) for k in om["kappa"]],
                      "x": [[float(c) for c in row] for row in om["x"]],
                      "v": [float(v) for v in om["v"]]}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--depth", type=int, default=0)
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--block", type=int, default=0, help="rollout workgroup (0: library choice)")
    ap.add_argument("--speculate", type=int, default=-1,
                    help="speculation depth with --no-autotune (-1: library default)")
    ap.add_argument("--mode-steps", type=int, default=0,
                    help="closed-loop steps timed for the Newton and FP64 search forms "
                         "(0: the same steps as the headline form)")
    ap.add_argument("--form", choices=["fp32_adjoint_newton", "fp64_sequential_bisection"],
                    default=None, help=argparse.SUPPRESS)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default schedule instead of the autotuned one")
    ap.add_argument("--tune-steps", type=int, default=50,
                    help="closed-loop updates the autotuner times each schedule on")
    ap.add_argument("--autotune-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-fc9", action="store_true",
                    help="skip the secondary 9-state grid-search measurement")
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
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration, "copies": 3}))
        return
    T = max(args.steps, args.warmup, args.tune_steps if args.autotune_only else 0)
    wl = W.workload_lq4_closed_loop(T=T)
    p = wl["problem"]
    r_seq = wl["r_seq"]
    prec = rg.PREC_F32_RECHECK if args.precision == "f32" else rg.PREC_F64
    x0 = np.asarray(wl["x0"], dtype=np.float64)
    if args.autotune_only:
        ga = rg.Governor(p, precision=prec, band=wl["band"], K=wl["K"], max_T=max(256, T))
        ga.set_step(0)
        print(json.dumps(ga.autotune(x0, wl["v_prev"], r_seq[: args.tune_steps])))
        ga.close()
        return

    # launch schedule (lanes per scenario, workgroup, search depth, first-round
    # prediction) from the autotuner, timed on the workload's first updates in a
    # child process of its own (its trial launches stay out of this process)
    tuned = None
    sched = dict(depth=args.depth, lanes=args.lanes, block=args.block)
    if args.speculate >= 0:
        sched["speculate"] = args.speculate
    if not args.no_autotune and args.tune_steps > 0:
        child = subprocess.run([sys.executable, os.path.abspath(__file__), "--autotune-only",
                                "--tune-steps", str(args.tune_steps)], capture_output=True, text=True)
        if child.returncode != 0:
            sys.stderr.write(child.stdout + child.stderr)
            raise SystemExit(f"autotuner failed (exit {child.returncode})")
        tuned = json.loads(child.stdout.strip().splitlines()[-1])
        sched = dict(depth=tuned["depth"], lanes=tuned["lanes"], block=tuned["block"],
                     predict=bool(tuned["predict"]), speculate=int(tuned["speculate"]))
    g = rg.Governor(p, precision=prec, band=wl["band"], K=wl["K"], max_T=max(256, T), **sched)

    # warmup: the first W updates of the workload (untimed)
    warm_launches = 0  # rollout launches of the warm-up (one per round, at least one per update)
    if args.warmup > 0:
        g.set_step(0)
        ow = g.closed_loop(x0, wl["v_prev"], r_seq[: args.warmup], use_graph=False)
        warm_launches = int(np.sum(np.maximum(1, np.asarray(ow["rounds"]))))

    # the workload's first K updates launched eagerly, with a HIP event pair
    # around every rollout launch (the roofline figure); untimed
    g.set_step(0)
    g.set_profiling(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out_e = g.closed_loop(x0, wl["v_prev"], r_seq[: args.steps], use_graph=False)
    torch.cuda.synchronize()
    elapsed_eager = time.perf_counter() - t1
    prof = g.profile()
    g.set_profiling(False)

    # timed region: the same K updates replayed from the captured HIP graphs of
    # generic search rounds (captured beforehand), from the initial state
    g.set_step(0)
    g.closed_loop(x0, wl["v_prev"], r_seq[:1], use_graph=True)
    g.set_step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = g.closed_loop(x0, wl["v_prev"], r_seq[: args.steps], use_graph=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    graph_same = bool(np.array_equal(out_e["v"], out["v"]))

    # The same closed loop under the other two search forms the metric names:
    # FP32 rollouts + adjoint-driven Newton, and plain sequential FP64 bisection
    # (one candidate per device round, Alg. 1 as written).  Each runs in a child
    # process over the same updates.
    modes = {}
    Km = min(args.steps, args.mode_steps) if args.mode_steps > 0 else args.steps
    for label in ["fp32_adjoint_newton", "fp64_sequential_bisection"]:
        child = subprocess.run([sys.executable, os.path.abspath(__file__), "--form", label,
                                "--steps", str(Km)], capture_output=True, text=True)
        if child.returncode != 0:
            sys.stderr.write(child.stdout + child.stderr)
            raise SystemExit(f"search form {label} failed (exit {child.returncode})")
        om = json.loads(child.stdout.strip().splitlines()[-1])
        kap = np.asarray(om.pop("kappa"))
        xs = np.asarray(om.pop("x"))
        vs = np.asarray(om.pop("v"))
        # accuracy at equal inputs: the headline bisection re-run at every state
        # of this form's own closed loop (its trajectory may leave the headline's
        # once a kappa differs within the 2^-K resolution)
        kb = np.zeros(Km)
        for s in range(Km):
            g.set_step(s)
            kb[s] = g.step(xs[s], r_seq[s], wl["v_prev"] if s == 0 else vs[s - 1])["kappa"]
        om["max_abs_kappa_diff_vs_bisection_same_state"] = float(np.max(np.abs(kap - kb)))
        om["kappa_within_2^-12"] = bool(np.all(np.abs(kap - kb) <= 2.0 ** -wl["K"] + 1e-15))
        om["same_closed_loop_as_headline"] = bool(np.array_equal(kap, out["kappa"][:Km]))
        modes[label] = om

    fc9 = {} if args.no_fc9 else fc9_grid_measurement(args)

    K = args.steps
    nominal = int(np.sum(out["bisect_passes"])) * p.N * p.H
    executed = int(np.sum(out["lane_steps"]))
    value = nominal / elapsed
    flops = prof["lane_steps"] * FLOP_PER_STEP_LQ4
    kern_s = prof["rollout_ms"] * 1e-3
    achieved = flops / kern_s / 1e12 if kern_s > 0 else 0.0
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
        "dtype": "f32" if prec == rg.PREC_F32_RECHECK else "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "plant": "LQ4", "N": p.N, "H": p.H, "dt": p.dt,
                   "K": wl["K"], "band": wl["band"], "rg_steps": K,
                   "precision": "fp32 rollouts + fp64 near-band recheck" if prec == 0 else "fp64",
                   "search": (f"bisection: first device round = kappa 1 probe + the midpoints on "
                              f"the path to the previous update's kappa, then "
                              f"{g.options.depth} levels per round" if g.options.predict else
                              f"bisection, {g.options.depth} levels per device round"),
                   "lanes_per_scenario": g.options.lanes,
                   "workgroup": g.options.block if g.options.block else 256,
                   "first_round_prediction": bool(g.options.predict),
                   "speculation_depth": int(g.options.speculate),
                   "schedule": ("autotuned on the first %d updates" % args.tune_steps
                                if tuned else "library default or command line"),
                   "launch": "captured HIP graphs of four generic search rounds, replayed until every update is recorded"},
        "rg_updates_per_s": K / elapsed,
        "executed_scenario_steps_per_s": executed / elapsed,
        "eager_profiled": {"ms_per_step": elapsed_eager / K * 1e3,
                           "rg_updates_per_s": K / elapsed_eager,
                           "value": nominal / elapsed_eager, "same_result": graph_same},
        "search_modes": dict(modes, fp32_speculative_bisection={
            "rg_updates_per_s": K / elapsed, "ms_per_step": elapsed / K * 1e3, "steps": K,
            "rounds_per_step": float(np.mean(out["rounds"]))}),
        "fc9_grid": fc9,
        "search_stats": {"rounds": int(np.sum(out["rounds"])),
                         "candidates": int(np.sum(out["candidates"])),
                         "rechecks": int(np.sum(out["rechecks"])),
                         "bisect_passes": int(np.sum(out["bisect_passes"])),
                         "infeasible_steps": int(np.sum(out["status"] != 0))},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic() if g.options.lanes == 4 else None,
                     "kernel": ("k_rollout_lq4_quad (one scenario per 4 lanes)" if g.options.lanes == 4
                                else "k_rollout<LQ4, float>"),
                     "launches": prof["rollout_launches"],
                     "launches_before": warm_launches,
                     "avg_launch_ms": prof["rollout_ms"] / max(1, prof["rollout_launches"]),
                     "flop_per_scenario_step": FLOP_PER_STEP_LQ4,
                     "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                     "achieved_hbm_gbs": prof["lane_steps"] * BYTES_PER_STEP_LQ4 / kern_s / 1e9
                     if kern_s > 0 else 0.0},
    }
    if not args.no_cpu_baseline:
        base, kappas = cpu_baseline(wl, r_seq, args.cpu_seconds)
        line["cpu_baseline"] = base
        n = len(kappas)
        line["cpu_baseline"]["kappa_agrees_first_updates"] = bool(
            np.all(np.abs(np.asarray(kappas) - out["kappa"][:n]) <= 2.0 ** -wl["K"]))
    g.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()

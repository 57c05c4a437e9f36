"""Writes lq4_closed_loop_n4096_h2000.txt: the FP64 oracle's closed loop of the
4-state bench workload (N = 4096 scenarios, H = 2000 RK4 steps of dt = 0.005,
200 RG updates, 12 bisection halvings after the kappa = 1 probe; Alg. 1 on the
robust verdict of Sec. II-C, true-plant steps as in Fig. 1).  It calls only the
oracle (test infrastructure); nothing here comes from the GPU library.

Run from the repository root:  python3 tests/golden/make_lq4_closed_loop_fixture.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2510_08288_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lq4_closed_loop_n4096_h2000.txt")


def main():
    wl = W.workload_lq4_closed_loop(T=200)
    p = wl["problem"]
    o = O.Oracle(p, nthreads=os.cpu_count() or 1)
    x = np.asarray(wl["x0"], dtype=np.float64)
    v_prev = wl["v_prev"]
    rows = []
    t0 = time.perf_counter()
    for s in range(wl["T"]):
        r = wl["r_seq"][s]
        res = o.bisect(x, r, v_prev, s, wl["K"])
        rows.append([s, r, v_prev, *x, res["kappa"], res["v"], res["passes"], res["status"]])
        x = o.plant_step(x, res["v"], s)
        v_prev = res["v"]
        print(f"update {s}: kappa {res['kappa']!r} passes {res['passes']} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle closed loop of lq4_closed_loop_n4096_h2000 (plant seed 24, scenario\n"
                "# seed 1234, eps 0.01, reference seed 2024): Alg. 1 with K = 12 on the robust\n"
                "# verdict (Sec. II-C), true plant as in Fig. 1.  Written by\n"
                "# make_lq4_closed_loop_fixture.py from the oracle alone.\n"
                "# columns: t r v_prev x0 x1 x2 x3 kappa v passes status (x, v_prev: state\n"
                "# and previous set-point the update starts from; floats in repr form)\n")
        for row in rows:
            f.write(" ".join(repr(float(c)) if i not in (0, 9, 10) else str(int(c))
                             for i, c in enumerate(row)) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()

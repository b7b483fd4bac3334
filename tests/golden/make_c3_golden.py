"""Writes tests/golden/c3_sampled.txt: oracle values of the 1872-DOF shell workload at full size.

Workload: the synthetic shell (12 x 24 triangle mesh, 6 DOF per node, 1872 DOF, half band 89),
d = 2, H = 20 (U~ = 41), S~ = 128 trajectories, S1 = 1024 average-acceleration Newmark steps
per period (App. E), omega_1 = 0.98 x the first natural frequency, omega_2 = omega_1 / sqrt(2),
initial iterate the linear harmonic response (fse_inputs.workload("C3")).

For the sampled trajectories TRAJ it records the terminal state zbar(2 pi) (Eqs. E4-E7, per-step
Newton to 1e-12) and the columns COLS of the sensitivity matrix Phi_s (Eqs. E8-E9), propagated
by the oracle's own recursion restricted to those columns.  Only oracle/ and the seeded input
builders are called.  Run from the repository root:

    python tests/golden/make_c3_golden.py          (about 20 minutes on 3 x 2 host threads)
"""
from __future__ import annotations

import os
import sys
import time
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(ROOT, "tests", "golden", "c3_sampled.txt")
TRAJ = [0, 45, 127]
COLS = [0, 900, 1871, 1972, 3743]


def one(s):
    from threadpoolctl import threadpool_limits
    from fse_inputs import workload
    from oracle import newmark, shooting
    with threadpool_limits(2):
        wl = workload("C3")
        tb = shooting.TorusTables(wl.torus)
        n = wl.system.n
        zbar0 = wl.initial_iterate(tb.table).reshape(2 * n, tb.U) @ tb.G.T
        t0 = time.time()
        out = newmark.integrate(wl.system, wl.omega, wl.torus.S1, tb.phases[:, s], zbar0[:, s],
                                sens=True, sens_cols=COLS)
        return s, out["zT"], out["Phi"], int(out["iters"].sum()), time.time() - t0


def main():
    with get_context("spawn").Pool(len(TRAJ)) as pool:
        res = sorted(pool.map(one, TRAJ))
    with open(OUT, "w") as f:
        f.write("# Oracle values of the 1872-DOF shell workload at full size (written by make_c3_golden.py).\n")
        f.write("# d = 2, H = 20, S~ = 128, S1 = 1024, omega from fse_inputs.workload('C3'), step tol 1e-12.\n")
        f.write(f"# trajectories {' '.join(map(str, TRAJ))}; Phi columns {' '.join(map(str, COLS))}\n")
        f.write("# per trajectory: a line 'traj s iters', then 2n lines 'zT  Phi[:, COLS]'\n")
        for s, zT, Phi, its, el in res:
            f.write(f"traj {s} {its}\n")
            for i in range(len(zT)):
                f.write(" ".join(f"{v:.17e}" for v in [zT[i], *Phi[i]]) + "\n")
            print(f"trajectory {s}: {its} step-Newton iterations, {el:.0f} s", flush=True)


if __name__ == "__main__":
    main()

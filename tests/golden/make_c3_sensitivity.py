"""Writes tests/golden/c3_sensitivity.txt: the floating-point conditioning of the 1872-DOF shell's
one-period map, measured on the oracle itself.

Trajectory 0 of the full-size shell workload (S1 = 1024) is integrated three times: as is, with
its initial state perturbed by a relative 1e-15 (seeded normal factors), and with omega_1 moved by
one unit in the last place.  Both perturbations are of the size of the rounding that any two FP64
implementations of the same steps make differently (summation order, fused multiply-adds, the
cosine of the forcing), so the relative change of zbar(2 pi) they cause is the scale below which
two correct implementations cannot be told apart.  The lumped masses of the rotational DOFs are
three orders of magnitude below those of the translations, and the consistent initial
acceleration divides by them.  Only oracle/ and the seeded input builders are called; run from
the repository root (about 20 minutes, three processes).
"""
from __future__ import annotations

import os
import sys
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(ROOT, "tests", "golden", "c3_sensitivity.txt")


def run(kind):
    from threadpoolctl import threadpool_limits
    from fse_inputs import workload
    from oracle import newmark, shooting
    with threadpool_limits(2):
        wl = workload("C3")
        tb = shooting.TorusTables(wl.torus)
        n = wl.system.n
        z0 = (wl.initial_iterate(tb.table).reshape(2 * n, tb.U) @ tb.G.T)[:, 0].copy()
        om = wl.omega.copy()
        if kind == "z0":
            z0 = z0 * (1.0 + 1e-15 * np.random.default_rng(0).normal(size=z0.size))
        elif kind == "omega":
            om[0] = np.nextafter(om[0], np.inf)
        return kind, newmark.integrate(wl.system, om, wl.torus.S1, tb.phases[:, 0], z0)["zT"]


def main():
    with get_context("spawn").Pool(3) as pool:
        res = dict(pool.map(run, ["base", "z0", "omega"]))
    base = res["base"]
    with open(OUT, "w") as f:
        f.write("# Relative change of zbar(2 pi) of trajectory 0 of the full-size shell (S1 = 1024) under\n")
        f.write("# rounding-sized perturbations, measured on the oracle (make_c3_sensitivity.py).\n")
        f.write("# columns: perturbation, ||zT' - zT|| / ||zT||\n")
        for k in ("z0", "omega"):
            f.write(f"{k} {np.linalg.norm(res[k] - base) / np.linalg.norm(base):.6e}\n")


if __name__ == "__main__":
    main()

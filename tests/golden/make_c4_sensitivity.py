"""Writes tests/golden/c4_sensitivity.txt: the floating-point conditioning of the one-period maps
of the trajectories that the eight-point three-frequency beam test samples, measured on the oracle
itself.

For each continuation point b (omega_1 = 36.5 ... 40 rad/s in 8 steps, omega = omega_1 (1, sqrt 2,
sqrt 3), linear harmonic start) trajectory (146 b) mod 1024 is integrated three times: as is, with
its initial state perturbed by a relative 1e-15 (seeded normal factors), and with omega_1 moved by
one unit in the last place.  Both perturbations are of the size of the rounding that two FP64
implementations of the same steps make differently, so the relative change of zbar(2 pi) they cause
is the scale below which two correct implementations cannot be told apart.  Only oracle/ and the
seeded input builders are called; run from the repository root (about half a minute).
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(ROOT, "tests", "golden", "c4_sensitivity.txt")


def main():
    from fse_inputs import workload
    from oracle import newmark, shooting
    rng = np.random.default_rng(0)
    rows = []
    for b, w1 in enumerate(np.linspace(36.5, 40.0, 8)):
        wl = workload("C4", omega1=float(w1))
        tb = shooting.TorusTables(wl.torus)
        n = wl.system.n
        s = (146 * b) % tb.Stilde
        z0 = (wl.initial_iterate(tb.table).reshape(2 * n, tb.U) @ tb.G.T)[:, s].copy()
        ph = tb.phases[:, s]
        base = newmark.integrate(wl.system, wl.omega, wl.torus.S1, ph, z0)["zT"]
        zp = newmark.integrate(wl.system, wl.omega, wl.torus.S1, ph,
                               z0 * (1.0 + 1e-15 * rng.normal(size=z0.size)))["zT"]
        om = wl.omega.copy()
        om[0] = np.nextafter(om[0], np.inf)
        wp = newmark.integrate(wl.system, om, wl.torus.S1, ph, z0)["zT"]
        nb = np.linalg.norm(base)
        rows.append((b, s, np.linalg.norm(zp - base) / nb, np.linalg.norm(wp - base) / nb))
        print(rows[-1], flush=True)
    with open(OUT, "w") as f:
        f.write("# point b, trajectory, relative change of zbar(2 pi) for a 1e-15 relative change of\n")
        f.write("# zbar(0), and for one ulp of omega_1 (oracle, make_c4_sensitivity.py)\n")
        for b, s, a, c in rows:
            f.write(f"{b} {s} {a:.3e} {c:.3e}\n")


if __name__ == "__main__":
    main()

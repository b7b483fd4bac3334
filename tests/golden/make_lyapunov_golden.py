"""Writes tests/golden/lyapunov_c2.txt and lyapunov_c4.txt: the oracle's Lyapunov exponents
(App. F, Eqs. F1-F3) of the 147-DOF von Karman beam at full size.

C2: d = 2, 64 trajectories, H = 15, S1 = 512, omega_1 = 40 rad/s; C4: d = 3, 32 x 32 = 1024
trajectories, H = 8 x 8, S1 = 512, omega_1 = 40 rad/s (fse_inputs.workload); both at their linear
harmonic initial iterate (the exponents are those of the quasi-periodic linearisation along the
trajectories that start there).  All trajectories are integrated with sensitivities (Eqs. E8-E9),
then N_Ly = 1000 Householder QR steps of the interpolated one-period maps with the identity as the
initial basis.  The same sweep is repeated from a start basis a rounding-sized step away from the
identity (the Q factor of I + 1e-14 N(0, 1), seeded), and the second column records, per exponent,
the change that makes.  The exponents of these maps span 6 ... -233 1/s over a period of 0.157 s,
so the product of the per-period maps spans far more than the FP64 range: the strongly
contracting directions, and the individual members of complex pairs and clusters, are set by
rounding and are not determined by any FP64 QR sweep (nor is their sum, the mean log|det Psi|,
which the smallest singular values dominate).  Only oracle/ and the seeded input builders are called.
Run from the repository root: python tests/golden/make_lyapunov_golden.py [--phi-cache DIR]
(about 15 minutes on 7 processes; with a cache directory the oracle's maps are kept there).
"""
from __future__ import annotations

import os
import sys
import time
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
N_LY = 1000


def _phi(args):
    name, s = args
    from threadpoolctl import threadpool_limits
    from fse_inputs import workload
    from oracle import shooting
    with threadpool_limits(1):
        wl = workload(name)
        tb = shooting.TorusTables(wl.torus)
        Z0 = wl.initial_iterate(tb.table)
        res = shooting.evaluate(wl.system, wl.torus, wl.omega, Z0, sens=True, tables=tb, samples=[s])
        return s, res["Phi"][s]


def main():
    from fse_inputs import workload
    from oracle import lyapunov, shooting
    cache = sys.argv[sys.argv.index("--phi-cache") + 1] if "--phi-cache" in sys.argv else None
    with get_context("spawn").Pool(7) as pool:
        for name in ("C2", "C4"):
            wl = workload(name)
            tb = shooting.TorusTables(wl.torus)
            t0 = time.time()
            path = os.path.join(cache, f"phi_{name.lower()}.npy") if cache else None
            if path and os.path.exists(path):
                Phi = np.load(path)
            else:
                out = pool.map(_phi, [(name, s) for s in range(tb.Stilde)], chunksize=4)
                Phi = np.stack([p for _, p in sorted(out, key=lambda x: x[0])])
                if path:
                    np.save(path, Phi)
            sig, srt, _ = lyapunov.exponents(Phi, wl.omega, tb, N_Ly=N_LY)
            n2 = Phi.shape[1]
            Q0, _ = np.linalg.qr(np.eye(n2) + 1e-14 * np.random.default_rng(0).normal(size=(n2, n2)))
            Q0 = Q0 * np.sign(np.diag(Q0))[None, :]
            sig1, _, _ = lyapunov.exponents(Phi, wl.omega, tb, N_Ly=N_LY, Q0=Q0)
            with open(os.path.join(ROOT, "tests", "golden", f"lyapunov_{name.lower()}.txt"), "w") as f:
                f.write(f"# Oracle Lyapunov exponents of workload {name} at its linear harmonic start, N_Ly = {N_LY},\n")
                f.write("# identity initial basis (make_lyapunov_golden.py); one per line in QR column order [1/s],\n")
                f.write("# then the change of that exponent when the start basis moves 1e-14 from the identity.\n")
                for v, v1 in zip(sig, sig1):
                    f.write(f"{v:.17e} {v1 - v:.3e}\n")
            print(name, f"{time.time() - t0:.0f} s", srt[:3], srt[-1], flush=True)


if __name__ == "__main__":
    main()

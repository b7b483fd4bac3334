"""FSE-Shooting in the hyper-time domain (oracle; test infrastructure only).

Sec. 3.4 of the paper writes the same shooting conditions with the trajectory initial
states themselves as unknowns: with zbar(0) the [2n][S~] samples of the initial torus,
    R(zbar(0), omega) = (I (x) Gamma R(rho) Gamma^-1) zbar(2 pi) - zbar(0)     (Eq. FSES_T),
where zbar(2 pi) are the states after one period of phi_1 (App. E, the same integrator).
The S~ x S~ operator A = Gamma R(rho) Gamma^-1 shifts the sampled torus by -2 pi rho through
its Fourier interpolant.  Its Jacobian is
    J[(i, s), (j, t)] = A[s, t] Phi_t[i, j] - delta,
with Phi_t the sensitivity matrix of trajectory t (Eqs. E8-E9).  Unknowns are ordered
state-major, (i, s) -> i S~ + s.  With unknown frequencies (d > e) the Newton step is bordered
by the columns dR/domega_u and the phase rows of Eq. (18) carried over through Z = Gamma^-1 zbar
(`border`), and the step also updates omega_u.

Pins (tests/test_oracle_hypertime.py): for zbar(0) = Gamma Z(0), the hyper-time residual is
Gamma applied to the multi-frequency residual (Gamma^-1 Gamma = I); the Jacobian against
central differences; a linear system's closed-form torus, sampled, solves it, and one Newton
step reaches it; on a nonlinear system the hyper-time Newton solution is the sampled
multi-frequency torus.  With unknown frequencies (border of `border`, a reading: the paper
gives this form no phase condition): with S~ = U~ the bordered step is Gamma times the
multi-frequency bordered step, and the border column matches central differences.
"""
from __future__ import annotations

import numpy as np

from . import newmark
from . import shooting
from . import torus as tor


def operator(tables, omega):
    """A = Gamma R(rho) Gamma^-1 (S~ x S~)."""
    omega = np.asarray(omega, dtype=float)
    Rm = tor.rotation(tables.table, omega[1:] / omega[0]) if tables.torus.d > 1 else np.eye(1)
    return tables.G @ Rm @ tables.Gi


def evaluate(sysm, torus, omega, zbar0, sens=False, tables=None, tol=1e-12, maxit=30):
    """Integrate every trajectory from the samples zbar0 [2n][S~]; returns zbarT, R, A and
    Phi [S~][2n][2n] if sens."""
    tb = tables or shooting.TorusTables(torus)
    omega = np.asarray(omega, dtype=float)
    z0 = np.asarray(zbar0, dtype=float)
    zT = np.empty_like(z0)
    Phi = np.empty((tb.Stilde, z0.shape[0], z0.shape[0])) if sens else None
    for s in range(tb.Stilde):
        out = newmark.integrate(sysm, omega, torus.S1, tb.phases[:, s], z0[:, s], sens=sens, tol=tol,
                                maxit=maxit, beta=getattr(torus, "beta", 0.25),
                                gamma=getattr(torus, "gamma", 0.5))
        zT[:, s] = out["zT"]
        if sens:
            Phi[s] = out["Phi"]
    A = operator(tb, omega)
    res = {"zbarT": zT, "A": A, "R": zT @ A.T - z0, "tables": tb}
    if sens:
        res["Phi"] = Phi
    return res


def jacobian(res):
    """J[(i, s), (j, t)] = A[s, t] Phi_t[i, j] - delta."""
    A, Phi = res["A"], res["Phi"]
    St, n2 = A.shape[0], Phi.shape[1]
    J4 = np.einsum("st,tij->isjt", A, Phi)
    J = J4.reshape(n2 * St, n2 * St)
    return J - np.eye(n2 * St)


def border(res, omega, e, zbar0):
    """Border of the Newton matrix for the unknown frequencies u = e+1..d (the paper gives the
    hyper-time form no phase condition; this carries Eqs. 18 and 23-24 over through
    Z = Gamma^-1 zbar): columns dR/d omega_u = (I (x) Gamma dR(rho)/d omega_u Gamma^-1) zbar(2 pi)
    and phase rows [(I (x) nabla_{phi_u}) Gamma^-1 zbar(0)]^T (I (x) Gamma^-1), as
    ([2n S~][d-e], [d-e][2n S~])."""
    tb = res["tables"]
    omega = np.asarray(omega, dtype=float)
    d = len(omega)
    z0 = np.asarray(zbar0, dtype=float)
    cols, rows = [], []
    for i in range(e + 1, d + 1):
        dA = tb.G @ tor.rotation_domega(tb.table, omega, i) @ tb.Gi
        cols.append((res["zbarT"] @ dA.T).ravel())
        pz = (z0 @ tb.Gi.T) @ tor.nabla(tb.table, i).T          # (I (x) nabla) Z(0), [2n][U~]
        rows.append((pz @ tb.Gi).ravel())                        # times (I (x) Gamma^-1)
    return np.array(cols).T, np.array(rows)


def newton_step(sysm, torus, omega, zbar0, tables=None, tol=1e-12):
    """zbar0 -> zbar0 - J^-1 R; returns (zbar_new, ||R||_2 before).  For d > e the unknowns are
    [zbar(0); omega_u] with the border of `border`; returns (zbar_new, omega_new, ||R||_2)."""
    res = evaluate(sysm, torus, omega, zbar0, sens=True, tables=tables, tol=tol)
    J = jacobian(res)
    if torus.d == torus.e:
        dz = np.linalg.solve(J, -res["R"].ravel())
        return zbar0 + dz.reshape(np.shape(zbar0)), float(np.linalg.norm(res["R"]))
    nu = torus.d - torus.e
    B, P = border(res, omega, torus.e, zbar0)
    big = np.block([[J, B], [P, np.zeros((nu, nu))]])
    x = np.linalg.solve(big, np.concatenate([-res["R"].ravel(), np.zeros(nu)]))
    om = np.array(omega, dtype=float)
    om[torus.e:] += x[-nu:]
    return np.asarray(zbar0, float) + x[:-nu].reshape(np.shape(zbar0)), om, float(np.linalg.norm(res["R"]))


def solve(sysm, torus, omega, zbar0, tol_R=1e-8, max_newton=20, tables=None):
    """Newton iterations until ||R||_2 < tol_R; returns (zbar0, history of ||R||_2), and for
    d > e (unknown frequencies, bordered step) (zbar0, omega, history)."""
    z = np.array(zbar0, dtype=float)
    om = np.array(omega, dtype=float)
    bordered = torus.d > torus.e
    hist = []
    for _ in range(max_newton):
        if bordered:
            z_new, om_new, r = newton_step(sysm, torus, om, z, tables=tables)
        else:
            z_new, r = newton_step(sysm, torus, om, z, tables=tables)
            om_new = om
        hist.append(r)
        if r < tol_R:
            return (z, om, hist) if bordered else (z, hist)
        z, om = z_new, om_new
    res = evaluate(sysm, torus, om, z, tables=tables)
    hist.append(float(np.linalg.norm(res["R"])))
    return (z, om, hist) if bordered else (z, hist)

"""Shooting residual, Jacobian and Newton step of FSE-Shooting (oracle; test infrastructure only).

The six steps of Sec. 3.3: Z(0) -> z(0, phi~) by the inverse DFT (Eq. 20),
every trajectory integrated independently (App. E), z(2 pi, phi~) -> Z(2 pi) by
the DFT (Eq. 21), rotation by R(rho) (Eq. 15) and the residual
R = (I (x) R(rho)) Z(2 pi) - Z(0) (Eq. 16).  The Jacobian is Eq. (22) and the
frequency derivatives Eqs. (23)-(24).  The Newton step solves the bordered
system of Eq. (17) (continuation variables [Z(0); omega_u]) with the proposed
phase condition of Eq. (18) taken with Z* = dZ (an orthogonality row).

Layout: Z is [2n][U~] (state-major, Eq. 10); zbar is [2n][S~] (App. D).

Pins (tests/test_oracle_shooting.py): the discrete closed-form linear torus
(R = 0, one Newton iteration), J = Phi (x) R - I for linear systems, central
finite differences of R in Z(0) and in omega, d = 1 reduction to classical
shooting.
"""
from __future__ import annotations

import numpy as np

from . import newmark
from . import torus as tor


class TorusTables:
    """Harmonic table, grid and AFT matrices of one torus discretisation."""

    def __init__(self, torus):
        self.torus = torus
        self.table = tor.harmonic_table(torus.K)
        self.U = tor.n_coefficients(torus.K)
        self.G, self.Gi = tor.gamma_matrices(self.table, torus.S) if torus.d > 1 else (
            np.ones((1, 1)), np.ones((1, 1)))
        self.phases = tor.sample_angles(torus.S) if torus.d > 1 else np.zeros((0, 1))
        self.Stilde = self.G.shape[0]


def evaluate(sysm, torus, omega, Z0, sens=False, omega_sens=False, tables=None,
             samples=None, tol=1e-12, maxit=30):
    """Run the AFT-TI-DFT pipeline (Eq. 19b).  `samples` restricts integration to a
    subset of trajectories (zT of the others is left NaN) for sampled parity."""
    tb = tables or TorusTables(torus)
    omega = np.asarray(omega, dtype=float)
    n = sysm.n
    Z0 = np.asarray(Z0, dtype=float).reshape(2 * n, tb.U)
    zbar0 = Z0 @ tb.G.T                         # Eq. (20): (I (x) Gamma) Z(0)
    zbarT = np.full_like(zbar0, np.nan)
    Phi = np.full((tb.Stilde, 2 * n, 2 * n), np.nan) if sens else None
    dzw = np.full((tb.Stilde, 2 * n, sysm.e), np.nan) if omega_sens else None
    iters = np.zeros((tb.Stilde, torus.S1), dtype=np.int64)
    sel = range(tb.Stilde) if samples is None else samples
    for s in sel:
        out = newmark.integrate(sysm, omega, torus.S1, tb.phases[:, s], zbar0[:, s],
                                sens=sens, omega_sens=omega_sens, tol=tol, maxit=maxit,
                                beta=getattr(torus, "beta", 0.25), gamma=getattr(torus, "gamma", 0.5))
        zbarT[:, s] = out["zT"]
        iters[s] = out["iters"]
        if sens:
            Phi[s] = out["Phi"]
        if omega_sens:
            dzw[s] = out["dz_domega"]
    res = {"zbar0": zbar0, "zbarT": zbarT, "iters": iters, "tables": tb}
    if samples is None:
        Z2 = zbarT @ tb.Gi.T                    # Eq. (21): (I (x) Gamma^-1) zbar(2 pi)
        Rm = tor.rotation(tb.table, omega[1:] / omega[0]) if torus.d > 1 else np.eye(1)
        Zhat = Z2 @ Rm.T                         # Eq. (15): (I (x) R(rho)) Z(2 pi)
        res.update(Z2pi=Z2, Zhat=Zhat, R=Zhat - Z0, Rrot=Rm)
    if sens:
        res["Phi"] = Phi
    if omega_sens:
        res["dzbar_domega"] = dzw
    return res


def jacobian(res, omega=None):
    """dR/dZ(0) of Eq. (22), entrywise:
    J[(i,l),(j,m)] = sum_s (R Gamma^-1)[l,s] Phi_s[i,j] Gamma[s,m] - delta.
    """
    tb = res["tables"]
    A = res["Rrot"] @ tb.Gi
    Phi = res["Phi"]
    n2 = Phi.shape[1]
    J4 = np.einsum("ls,sij,sm->iljm", A, Phi, tb.G, optimize=True)
    J = J4.reshape(n2 * tb.U, n2 * tb.U)
    J -= np.eye(n2 * tb.U)
    return J


def jacobian_kron(res):
    """Eq. (22) literally with Kronecker products (small cases only)."""
    tb = res["tables"]
    Phi = res["Phi"]
    St = tb.Stilde
    n2 = Phi.shape[1]
    big = np.zeros((n2 * St, n2 * St))
    for s in range(St):
        o = np.zeros((St, St))
        o[s, s] = 1.0
        big += np.kron(Phi[s], o)                # Eq. (E9)
    left = np.kron(np.eye(n2), res["Rrot"] @ tb.Gi)
    right = np.kron(np.eye(n2), tb.G)
    return left @ big @ right - np.eye(n2 * tb.U)


def residual_domega(res, omega, e, first=1):
    """dR/d omega_i of Eq. (23), i = first..d, as a (2n U~) x (d - first + 1) matrix.

    For i <= e the trajectory term needs res['dzbar_domega'] (integrated with
    omega_sens=True); for i > e only the rotation term is present.
    """
    tb = res["tables"]
    omega = np.asarray(omega, dtype=float)
    d = len(omega)
    n2 = res["Z2pi"].shape[0]
    out = np.zeros((n2 * tb.U, d - first + 1))
    A = res["Rrot"] @ tb.Gi
    for i in range(first, d + 1):
        dR = tor.rotation_domega(tb.table, omega, i)
        col = res["Z2pi"] @ dR.T
        if i <= e:
            dz = res["dzbar_domega"][:, :, i - 1].T      # [2n][S~]
            col = col + dz @ A.T
        out[:, i - first] = col.ravel()
    return out


def phase_rows(tables, Z0, e, d):
    """Rows of the proposed phase condition, Eq. (18) with Z* = dZ:
    [(I (x) nabla_{phi_i}) Z(0)]^T dZ = 0 for the unknown frequencies i = e+1..d."""
    rows = []
    for i in range(e + 1, d + 1):
        Nb = tor.nabla(tables.table, i)
        rows.append((Z0 @ Nb.T).ravel())
    return np.array(rows).reshape(d - e, -1)


def newton_step(sysm, torus, omega, Z0, tables=None, tol=1e-12):
    """One Newton-Raphson update of [Z(0); omega_u] (Sec. 3.3 step 6).

    For d = e all frequencies are fixed (frequency conditions FC_j hold exactly,
    Eq. 17b) and the step is dZ = -J^-1 R.  For d > e the unknown frequencies
    omega_{e+1..d} are added with the phase rows of Eq. (18).
    Returns (Z_new, omega_new, ||R||_2 before the update).
    """
    tb = tables or TorusTables(torus)
    d, e = torus.d, torus.e
    res = evaluate(sysm, torus, omega, Z0, sens=True, omega_sens=False, tables=tb, tol=tol)
    J = jacobian(res)
    R = res["R"].ravel()
    if d == e:
        dZ = np.linalg.solve(J, -R)
        return Z0 + dZ.reshape(Z0.shape), np.array(omega, float), float(np.linalg.norm(R))
    dRw = residual_domega(res, omega, e, first=e + 1)
    P = phase_rows(tb, Z0, e, d)
    nu = d - e
    big = np.block([[J, dRw], [P, np.zeros((nu, nu))]])
    rhs = np.concatenate([-R, np.zeros(nu)])
    x = np.linalg.solve(big, rhs)
    om = np.array(omega, float)
    om[e:] += x[-nu:]
    return Z0 + x[:-nu].reshape(Z0.shape), om, float(np.linalg.norm(R))


def solve(sysm, torus, omega, Z0, tol_R=1e-8, max_newton=20, tables=None, step_tol=1e-12):
    """Newton iterations until ||R||_2 < tol_R (App. C stopping rule).  Returns
    (Z, omega, history of ||R||_2)."""
    tb = tables or TorusTables(torus)
    Z = np.array(Z0, float)
    om = np.array(omega, float)
    hist = []
    for _ in range(max_newton):
        res = evaluate(sysm, torus, om, Z, tables=tb, tol=step_tol)
        r = float(np.linalg.norm(res["R"]))
        hist.append(r)
        if r < tol_R:
            return Z, om, hist
        Z, om, _ = newton_step(sysm, torus, om, Z, tables=tb, tol=step_tol)
    res = evaluate(sysm, torus, om, Z, tables=tb, tol=step_tol)
    hist.append(float(np.linalg.norm(res["R"])))
    return Z, om, hist

"""Multiple FSE-Shooting (oracle; test infrastructure only).

The paper recommends a multiple FSE-Shooting method for robustness and a larger convergence
domain (Sec. 5, first recommendation) without giving its form; this is the classical
multiple-shooting reading of Sec. 3.  The period of phi_1 is cut into M segments of S1/M
Newmark steps.  The unknowns are the M sections of the torus at phi_1 = 2 pi m / M,
Z^(m) [2n][U~] in the basis of Eq. (13) over the phases phi~ of the other frequencies at
that moment.  Segment m integrates the trajectories that start on section m at the grid
phases phi~_s (inverse DFT, Eq. 20), with the forcing of frequency 1 starting at phase
2 pi m / M (the others at phi_{i,s}, Eq. E1).  After 2 pi / M of phi_1 they reach phases
phi~_s + 2 pi rho / M, so invariance gives, as Eq. (16) does for the whole period,
    R_m = (I (x) R(rho / M)) Gamma^-1 zbar^(m)(2 pi / M) - Z^((m + 1) mod M),
and M = 1 is FSE-Shooting itself.  The Jacobian is block-cyclic: d R_m / d Z^(m) is the
Eq. (22) operator of segment m without its identity, d R_m / d Z^(m+1) = -I.

Pins (tests/test_oracle_multiple.py): M = 1 equals the single-shooting residual and
Jacobian; on a linear system one Newton step lands on the closed-form discrete torus, whose
section m is the section-0 torus with the harmonic of frequency 1 turned by 2 pi m / M;
central finite differences of R; on a nonlinear system the converged section 0 agrees with
the single-shooting torus to the Fourier truncation.  With unknown frequencies (d > e):
M = 1 gives the single-shooting bordered step, dR/d omega_u matches central differences, and
the forced van der Pol torus from two segments has the single-shooting free frequency.
"""
from __future__ import annotations

import math

import numpy as np

from . import newmark
from . import shooting
from . import torus as tor


def evaluate(sysm, torus, omega, Zs, M, sens=False, tables=None, tol=1e-12, maxit=30):
    """Zs [M][2n][U~] -> residual R [M][2n][U~] (and Phi [M][S~][2n][2n] if sens)."""
    if torus.S1 % M:
        raise ValueError("S1 must be a multiple of the number of segments")
    tb = tables or shooting.TorusTables(torus)
    omega = np.asarray(omega, dtype=float)
    n = sysm.n
    Zs = np.asarray(Zs, dtype=float).reshape(M, 2 * n, tb.U)
    steps = torus.S1 // M
    Rm = tor.rotation(tb.table, omega[1:] / omega[0] / M) if torus.d > 1 else np.eye(1)
    R = np.empty_like(Zs)
    Phi = np.empty((M, tb.Stilde, 2 * n, 2 * n)) if sens else None
    for m in range(M):
        zbar0 = Zs[m] @ tb.G.T
        zbarT = np.empty_like(zbar0)
        for s in range(tb.Stilde):
            out = newmark.integrate(sysm, omega, torus.S1, tb.phases[:, s], zbar0[:, s], sens=sens, tol=tol,
                                    maxit=maxit, beta=getattr(torus, "beta", 0.25),
                                    gamma=getattr(torus, "gamma", 0.5), steps=steps,
                                    phi0=2.0 * math.pi * m / M)
            zbarT[:, s] = out["zT"]
            if sens:
                Phi[m, s] = out["Phi"]
        R[m] = (zbarT @ tb.Gi.T) @ Rm.T - Zs[(m + 1) % M]
    res = {"R": R, "Rrot": Rm, "tables": tb, "M": M}
    if sens:
        res["Phi"] = Phi
    return res


def jacobian(res):
    """Block-cyclic dR/dZ, unknowns ordered [Z^(0); ...; Z^(M-1)], each state-major."""
    tb, M, Phi = res["tables"], res["M"], res["Phi"]
    n2 = Phi.shape[2]
    N = n2 * tb.U
    A = res["Rrot"] @ tb.Gi
    J = np.zeros((M * N, M * N))
    for m in range(M):
        blk = np.einsum("ls,sij,sk->iljk", A, Phi[m], tb.G, optimize=True).reshape(N, N)
        J[m * N:(m + 1) * N, m * N:(m + 1) * N] += blk
        m1 = (m + 1) % M
        J[m * N:(m + 1) * N, m1 * N:(m1 + 1) * N] -= np.eye(N)
    return J


def residual_domega_u(res, omega, e, Zs):
    """dR/d omega_u for the unknown base frequencies u = e+1..d, as [M 2n U~][d-e].

    The trajectories do not depend on an unknown frequency (only forcing frequencies enter
    Eq. E1); it acts through the rotation R(rho / M) alone: d R_m / d omega_u =
    (I (x) dR(rho/M)/d omega_u) Gamma^-1 zbar^(m)(2 pi / M), where R_m + Z^(m+1) is
    R(rho/M) Gamma^-1 zbar^(m)(2 pi / M).  With omega' = (omega_1, omega_2 / M, ...),
    R(rho/M) = R(rho') and dR(rho/M)/d omega_u = (1/M) dR(rho')/d omega'_u (Eq. 24)."""
    tb, M = res["tables"], res["M"]
    omega = np.asarray(omega, dtype=float)
    d = len(omega)
    om_s = np.concatenate([omega[:1], omega[1:] / M])
    Zs = np.asarray(Zs, dtype=float).reshape(res["R"].shape)
    Zend = np.stack([np.linalg.solve(res["Rrot"], (res["R"][m] + Zs[(m + 1) % M]).T).T for m in range(M)])
    cols = []
    for i in range(e + 1, d + 1):
        dR = tor.rotation_domega(tb.table, om_s, i) / M
        cols.append(np.concatenate([(Zend[m] @ dR.T).ravel() for m in range(M)]))
    return np.array(cols).T


def newton_step(sysm, torus, omega, Zs, M, tables=None):
    """Zs -> Zs - J^-1 R; returns (Zs_new, ||R||_2 before).  For d > e the unknowns are
    [Z^(0..M-1); omega_u], bordered as in single shooting (Eqs. 17-18) by the columns
    dR/d omega_u and the phase rows of Eq. (18) on section 0; returns (Zs_new, omega_new,
    ||R||_2 before) then."""
    res = evaluate(sysm, torus, omega, Zs, M, sens=True, tables=tables)
    d, e = torus.d, torus.e
    if d == e:
        dz = np.linalg.solve(jacobian(res), -res["R"].ravel())
        return np.asarray(Zs, dtype=float) + dz.reshape(res["R"].shape), float(np.linalg.norm(res["R"]))
    J = jacobian(res)
    nu = d - e
    B = residual_domega_u(res, omega, e, Zs)
    P = np.zeros((nu, J.shape[0]))
    P[:, :res["R"][0].size] = shooting.phase_rows(res["tables"], np.asarray(Zs, dtype=float)[0], e, d)
    big = np.block([[J, B], [P, np.zeros((nu, nu))]])
    x = np.linalg.solve(big, np.concatenate([-res["R"].ravel(), np.zeros(nu)]))
    om = np.array(omega, dtype=float)
    om[e:] += x[-nu:]
    return (np.asarray(Zs, dtype=float) + x[:-nu].reshape(res["R"].shape), om,
            float(np.linalg.norm(res["R"])))


def solve(sysm, torus, omega, Zs, M, tol_R=1e-8, max_newton=20, tables=None):
    """Newton iterations until ||R||_2 < tol_R; returns (Zs, history of ||R||_2), or
    (Zs, omega, history) when d > e."""
    Z = np.array(Zs, dtype=float)
    om = np.array(omega, dtype=float)
    bordered = torus.d > torus.e
    hist = []
    for _ in range(max_newton):
        if bordered:
            Zn, omn, r = newton_step(sysm, torus, om, Z, M, tables=tables)
        else:
            Zn, r = newton_step(sysm, torus, om, Z, M, tables=tables)
        hist.append(r)
        if r < tol_R:
            return (Z, om, hist) if bordered else (Z, hist)
        Z = Zn
        if bordered:
            om = omn
    hist.append(float(np.linalg.norm(evaluate(sysm, torus, om, Z, M, tables=tables)["R"])))
    return (Z, om, hist) if bordered else (Z, hist)

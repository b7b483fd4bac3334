"""Pseudo-arclength continuation in omega_1 (oracle; test infrastructure only).

App. C of the paper: at a known solution (chi_j, p_j) the tangent solves Eq. (C1),
the next point is predicted along it (Eq. C2) and corrected by Newton iterations
constrained orthogonal to the tangent (Eq. C3).  The continuation problem is the
one of Sec. 3.2.1 with p = omega_1: the unknowns are chi = [Z(0); omega_u]
(omega_u = omega_{e+1..d}, closed by the phase rows of Eq. 18), the forcing
frequencies follow omega_1 through the frequency conditions omega_j = rho_j
omega_1 (j = 2..e, rho_j fixed), so that the extended residual is
F(chi, p) = [R(Z(0), omega); phase rows].

Readings where the paper is silent or loose:
  * the tangent is normalised to unit 2-norm over [chi; p] (the printed
    normalisation by |dp| breaks down at a fold, where dp = 0);
  * the first tangent has no predecessor: its last row is e_p, oriented by the
    sign of the step, i.e. the tangent of the curve solved for dchi with dp = 1;
  * step control: a corrector that has not reached ||R||_2 < tol in maxit
    iterations (or whose integration fails) is restarted from the same point with
    half the step, at most 6 times; the step after an accepted one is doubled
    back, never beyond the requested step.

Pins (tests/test_oracle_continuation.py): dR/dp against central differences along
the frequency conditions; on a linear system every point of the path is the
closed-form discrete torus at its omega_1; on a forced Duffing oscillator the
path turns at the folds of the resonance curve, where the determinant of dR/dZ
changes sign; the corrector lands on the hyperplane t_j^T (x - x_j) = s.
"""
from __future__ import annotations

import numpy as np

from . import newmark
from . import shooting


def frequencies(omega_ref, p, e):
    """omega along the path: omega_1 = p, omega_j = (omega_ref_j / omega_ref_1) p for
    the forcing frequencies j = 2..e (frequency conditions), the unknown frequencies
    omega_{e+1..d} as given in omega_ref."""
    om = np.array(omega_ref, dtype=float)
    rho = om[:e] / om[0]
    om[:e] = rho * p
    return om


def residual_dp(res, omega, e):
    """dR/dp for p = omega_1 with the frequency conditions omega_j = rho_j omega_1
    (j = 2..e) and the unknown frequencies held: the chain rule over the columns
    of Eq. (23), dR/dp = dR/domega_1 + sum_{j=2..e} rho_j dR/domega_j."""
    omega = np.asarray(omega, dtype=float)
    cols = shooting.residual_domega(res, omega, e, first=1)
    out = cols[:, 0].copy()
    for j in range(2, e + 1):
        out += omega[j - 1] / omega[0] * cols[:, j - 1]
    return out


def extended_system(sysm, torus, omega, Z0, tables, tol=1e-12):
    """F = [R; 0] and its Jacobian A = [[J, dR/domega_u, dR/dp], [P, 0, 0]] at
    (Z0, omega), with the phase rows P of Eq. (18) (d > e only).  Columns are
    ordered [Z(0) (2n U~), omega_u (d - e), p]."""
    d, e = torus.d, torus.e
    res = shooting.evaluate(sysm, torus, omega, Z0, sens=True, omega_sens=True, tables=tables,
                            tol=tol)
    J = shooting.jacobian(res)
    N = J.shape[0]
    nu = d - e
    A = np.zeros((N + nu, N + nu + 1))
    A[:N, :N] = J
    if nu > 0:
        A[:N, N:N + nu] = shooting.residual_domega(res, omega, e, first=e + 1)
        A[N:, :N] = shooting.phase_rows(tables, Z0, e, d)
    A[:N, N + nu] = residual_dp(res, omega, e)
    F = np.concatenate([res["R"].ravel(), np.zeros(nu)])
    return F, A


def tangent(A, t_prev):
    """Eq. (C1): [A; t_prev^T] t = [0; 1], then unit 2-norm.  The last row keeps the
    orientation of t_prev (t_prev^T t > 0)."""
    M = np.vstack([A, t_prev])
    rhs = np.zeros(M.shape[0])
    rhs[-1] = 1.0
    t = np.linalg.solve(M, rhs)
    return t / np.linalg.norm(t)


def _unpack(x, omega_ref, N, e, shape):
    """x = [Z(0); omega_u; p] -> (Z0, omega)."""
    nu = len(omega_ref) - e
    om = frequencies(omega_ref, x[-1], e)
    om[e:] = x[N:N + nu]
    return x[:N].reshape(shape), om


def _pack(Z0, omega, e):
    return np.concatenate([np.ravel(Z0), np.asarray(omega, float)[e:], [omega[0]]])


def corrector(sysm, torus, omega_ref, x_pred, t, tables, tol_R, maxit, shape):
    """Newton iterations of Eq. (C3) from the prediction x_pred, every correction
    orthogonal to t.  Returns (x, A, ||R||_2 history) or None if ||R||_2 < tol_R is
    not reached in maxit corrections (or an integration fails)."""
    e = torus.e
    N = int(np.prod(shape))
    x = x_pred.copy()
    hist = []
    try:
        for k in range(maxit + 1):
            Z0, om = _unpack(x, omega_ref, N, e, shape)
            F, A = extended_system(sysm, torus, om, Z0, tables)
            r = float(np.linalg.norm(F[:N]))
            hist.append(r)
            if r < tol_R:
                return x, A, hist
            if k == maxit or not np.isfinite(r):
                return None
            M = np.vstack([A, t])
            dx = np.linalg.solve(M, -np.concatenate([F, [0.0]]))
            x = x + dx
    except (newmark.StepNewtonError, np.linalg.LinAlgError):
        return None
    return None


def arclength(sysm, torus, omega0, Z0, ds, npts, tables=None, tol_R=1e-10, maxit=8,
              max_halvings=6):
    """Trace npts points of the branch through the converged solution (Z0, omega0)
    with step ds in the 2-norm of [Z(0); omega_u; omega_1] (ds > 0: omega_1
    increasing at the start).  Returns a list of dicts with Z, omega, tangent t,
    step s taken, corrector history and the prediction x_pred (None for point 0)."""
    tb = tables or shooting.TorusTables(torus)
    e = torus.e
    Z0 = np.asarray(Z0, dtype=float)
    shape = Z0.shape
    N = Z0.size
    x = _pack(Z0, omega0, e)
    F, A = extended_system(sysm, torus, omega0, Z0, tb)
    t0 = np.zeros(x.size)
    t0[-1] = 1.0 if ds > 0 else -1.0
    t = tangent(A, t0)
    out = [{"Z": Z0.copy(), "omega": np.array(omega0, float), "t": t, "s": 0.0,
            "hist": [float(np.linalg.norm(F[:N]))], "x_pred": None}]
    s_max = abs(ds)
    s = s_max
    while len(out) < npts:
        got = None
        for _ in range(max_halvings + 1):
            x_pred = x + s * t
            got = corrector(sysm, torus, omega0, x_pred, t, tb, tol_R, maxit, shape)
            if got is not None:
                break
            s *= 0.5
        if got is None:
            raise RuntimeError(f"arclength corrector failed after {max_halvings} halvings "
                               f"at point {len(out)}")
        x_new, A, hist = got
        t = tangent(A, t)
        Zn, om = _unpack(x_new, omega0, N, e, shape)
        out.append({"Z": Zn, "omega": om, "t": t, "s": s, "hist": hist, "x_pred": x_pred})
        x = x_new
        s = min(2.0 * s, s_max)
    return out

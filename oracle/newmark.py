"""Newmark integration of one trajectory with sensitivities (oracle; test infrastructure only).

Follows App. E of the paper: the trajectory ODE (Eq. E1/E2)
    omega_1^2 M a + omega_1 D u + K q + f_nl(q) - e = 0,   u = q', a = q''  (' = d/dphi_1)
is stepped with the average-acceleration rule (Eqs. E4-E5); every step solves
Eq. (E6) S q_{k+1} + f_nl(q_{k+1}) = b_k (Eq. E7) by full-tangent Newton, and
the sensitivities d[q;u](2pi)/d[q;u](0) (Eq. E8) are the exact derivative of
the converged discrete map.

Readings where the paper is silent:
  * the state is [q; u] with u = dq/dphi_1 (App. E), not [q; qdot];
  * a_0 is the acceleration consistent with the equation of motion at phi_1 = 0;
  * Newton predictor q_k + D u_k + D^2/2 a_k; stop when ||dq||_inf <= tol *
    max(||q||_inf, q_scale), or when the update stops shrinking while already
    below 1e3 tol (the FP64 noise floor); at most `maxit` iterations;
  * the "adjoint system" of App. E is read as the variational (sensitivity) system;
  * f_nl may depend on qdot = omega_1 u (Eq. 1 allows it; the paper's examples do not):
    a tensor factor index in [n, 2n) names qdot.  Its tangent C_t = d f_nl / d qdot adds
    omega_1 gamma/(beta h) C_t to the step's iteration matrix and enters the
    sensitivities as the state-dependent damping D + C_t (general rule only);
  * nonsmooth forces (the paper recommends the extension without giving one) are read as
    unilateral penalty contacts, piecewise linear in q: the step Newton uses the generalised
    derivative (contact closed iff s q_i - g > 0), and the sensitivities are the derivative of
    the discrete map wherever no step lands exactly on a gap (almost everywhere).

Pins (tests/test_oracle_newmark.py): the closed-form average-acceleration
response of an undamped oscillator (unit amplitude, phase 2 atan(Omega h/2) per
step), discrete energy conservation, the discrete linear steady state, and
central finite differences of the sensitivities and of the omega-derivatives;
with velocity-dependent forces (tests/test_oracle_velocity.py) finite differences
of the sensitivities and of both tangents, and the forced van der Pol torus against
the averaging result (limit-cycle frequency 1 - mu^2/16, amplitude 2) and its
Lyapunov exponents (one zero, one near -mu); with unilateral contacts
(tests/test_oracle_contact.py) the step equation solved by its case split, open contacts
changing nothing, finite differences of the sensitivities, second-order convergence of the
impact orbit to the exact piecewise flow, the orbit as the end of a long transient, and the
half-wave symmetry of two symmetric stops.
"""
from __future__ import annotations

import math

import numpy as np


class StepNewtonError(RuntimeError):
    pass


def has_velocity(sysm) -> bool:
    """Forces that depend on qdot: a tensor factor index in [n, 2n) names qdot_{index - n}
    (the f_nl(q, qdot) of Eq. 1; the paper's examples depend on q only)."""
    n = sysm.n
    return bool((len(sysm.t2_val) and sysm.t2_idx[:, 1:].max() >= n)
                or (len(sysm.t3_val) and sysm.t3_idx[:, 1:].max() >= n))


def has_contact(sysm) -> bool:
    return len(getattr(sysm, "con_k", ())) > 0


def contact_force(sysm, q: np.ndarray) -> np.ndarray:
    """Unilateral penalty contacts, a nonsmooth f_nl (the paper's third recommendation): contact c
    on DOF i with direction s = +-1, gap g and stiffness k pushes back with s k max(s q_i - g, 0)."""
    f = np.zeros(len(q))
    for i, sg, g, k in zip(sysm.con_dof, sysm.con_dir, sysm.con_gap, sysm.con_k):
        f[i] += sg * k * max(sg * q[i] - g, 0.0)
    return f


def contact_tangent(sysm, q: np.ndarray) -> np.ndarray:
    """Generalised derivative of contact_force: k on the diagonal of a closed contact
    (s q_i - g > 0); an open contact or one exactly at its gap contributes nothing."""
    Kt = np.zeros((len(q), len(q)))
    for i, sg, g, k in zip(sysm.con_dof, sysm.con_dir, sysm.con_gap, sysm.con_k):
        if sg * q[i] - g > 0.0:
            Kt[i, i] += k
    return Kt


def _y(q, qd):
    return q if qd is None else np.concatenate([q, qd])


def internal_force(sysm, q: np.ndarray, qd: np.ndarray = None) -> np.ndarray:
    """f_nl(q, qdot)_i = sum t2 y_j y_k + sum t3 y_j y_k y_l, y = [q; qdot]."""
    n = len(q)
    y = _y(q, qd)
    f = np.zeros(n)
    if len(sysm.t2_val):
        i, j, k = sysm.t2_idx.T
        f += np.bincount(i, weights=sysm.t2_val * y[j] * y[k], minlength=n)
    if len(sysm.t3_val):
        i, j, k, l = sysm.t3_idx.T
        f += np.bincount(i, weights=sysm.t3_val * y[j] * y[k] * y[l], minlength=n)
    if has_contact(sysm):
        f += contact_force(sysm, q)
    return f


def tangents(sysm, q: np.ndarray, qd: np.ndarray = None):
    """(K_t, C_t) = (d f_nl / d q, d f_nl / d qdot), dense n x n each."""
    n = len(q)
    y = _y(q, qd)
    G = np.zeros((n, len(y)))
    if len(sysm.t2_val):
        i, j, k = sysm.t2_idx.T
        v = sysm.t2_val
        np.add.at(G, (i, j), v * y[k])
        np.add.at(G, (i, k), v * y[j])
    if len(sysm.t3_val):
        i, j, k, l = sysm.t3_idx.T
        v = sysm.t3_val
        np.add.at(G, (i, j), v * y[k] * y[l])
        np.add.at(G, (i, k), v * y[j] * y[l])
        np.add.at(G, (i, l), v * y[j] * y[k])
    Kt = G[:, :n] + (contact_tangent(sysm, q) if has_contact(sysm) else 0.0)
    return Kt, (G[:, n:] if qd is not None else np.zeros((n, n)))


def tangent(sysm, q: np.ndarray) -> np.ndarray:
    """K_t(q) = d f_nl / d q (dense; forces of q only)."""
    n = len(q)
    Kt = np.zeros((n, n))
    if len(sysm.t2_val):
        i, j, k = sysm.t2_idx.T
        v = sysm.t2_val
        np.add.at(Kt, (i, j), v * q[k])
        np.add.at(Kt, (i, k), v * q[j])
    if len(sysm.t3_val):
        i, j, k, l = sysm.t3_idx.T
        v = sysm.t3_val
        np.add.at(Kt, (i, j), v * q[k] * q[l])
        np.add.at(Kt, (i, k), v * q[j] * q[l])
        np.add.at(Kt, (i, l), v * q[j] * q[k])
    if has_contact(sysm):
        Kt += contact_tangent(sysm, q)
    return Kt


def forcing(sysm, omega, phases, phi1: float, phi0: float = 0.0) -> np.ndarray:
    """e(phi_1, phi^_s + rho^ phi_1) of Eq. (E1).

    Forcing i = 1 has argument phi0 + phi_1; forcing i = 2..e has phi_{i,s} + rho_i phi_1
    (phi0 = 0 on the section phi_1 = 0; a segment of multiple shooting starts at phi0).
    """
    e = sysm.F[0] * math.cos(phi0 + phi1)
    for i in range(2, sysm.e + 1):
        rho_i = omega[i - 1] / omega[0]
        e = e + sysm.F[i - 1] * math.cos(phases[i - 2] + rho_i * phi1)
    return e


def forcing_domega(sysm, omega, phases, phi1: float, i: int) -> np.ndarray:
    """d e / d omega_i (1-based i) through rho_j = omega_j / omega_1."""
    out = np.zeros(sysm.n)
    for j in range(2, sysm.e + 1):
        arg = phases[j - 2] + omega[j - 1] / omega[0] * phi1
        if i == 1:
            dr = -omega[j - 1] / omega[0] ** 2
        elif i == j:
            dr = 1.0 / omega[0]
        else:
            continue
        out = out - sysm.F[j - 1] * math.sin(arg) * dr * phi1
    return out


def _solve(A, B):
    return np.linalg.solve(A, B)


def integrate(sysm, omega, S1: int, phases, z0, sens: bool = False,
              omega_sens: bool = False, tol: float = 1e-12, maxit: int = 30,
              q_scale: float = 0.0, history: bool = False, beta: float = 0.25, gamma: float = 0.5,
              general: bool = False, steps: int = None, phi0: float = 0.0, sens_cols=None):
    """Integrate one trajectory from phi_1 = 0 to 2 pi in S1 Newmark steps.

    Returns dict with zT = [q; u](2 pi), Phi (2n x 2n) if sens, dz_domega
    (2n x e) if omega_sens, iters (Newton iterations per step), q_hist if history.
    (beta, gamma) other than the average-acceleration (1/4, 1/2) of App. E, or general=True,
    take the general Newmark rule (integrate_general).  steps < S1 integrates that many
    steps of h = 2 pi / S1 from the section phi_1 = phi0 (a segment of multiple shooting).
    sens_cols (average-acceleration rule): propagate only those columns of the sensitivities,
    Phi[:, sens_cols] (2n x len), by the same recursion started from the same columns of
    Q_0, U_0, A_0 (the recursion is linear and acts on every column on its own).
    """
    if general or beta != 0.25 or gamma != 0.5 or has_velocity(sysm):
        if sens_cols is not None:
            raise ValueError("sens_cols needs the average-acceleration rule")
        return integrate_general(sysm, omega, S1, phases, z0, sens=sens, omega_sens=omega_sens, tol=tol,
                                 maxit=maxit, q_scale=q_scale, history=history, beta=beta, gamma=gamma,
                                 steps=steps, phi0=phi0)
    steps = S1 if steps is None else steps
    M, D, K = sysm.M, sysm.D, sysm.K
    n = sysm.n
    omega = np.asarray(omega, dtype=float)
    w1 = omega[0]
    h = 2.0 * math.pi / S1
    c0, c1, c2 = 4.0 / h ** 2, 4.0 / h, 2.0 / h
    S = w1 ** 2 * c0 * M + w1 * c2 * D + K
    q = np.array(z0[:n], dtype=float)
    u = np.array(z0[n:], dtype=float)
    Mw = w1 ** 2 * M
    a = _solve(Mw, forcing(sysm, omega, phases, 0.0, phi0) - w1 * D @ u - K @ q
               - internal_force(sysm, q))
    if sens:
        Q = np.hstack([np.eye(n), np.zeros((n, n))])
        U = np.hstack([np.zeros((n, n)), np.eye(n)])
        A = -_solve(Mw, np.hstack([K + tangent(sysm, q), w1 * D]))
        if sens_cols is not None:
            cols = np.asarray(sens_cols, dtype=np.int64)
            Q, U, A = Q[:, cols], U[:, cols], A[:, cols]
    ne = sysm.e
    if omega_sens:
        # d q0/d omega = d u0/d omega = 0; d a0/d omega_i from the consistency equation
        Qw = np.zeros((n, ne))
        Uw = np.zeros((n, ne))
        Aw = np.zeros((n, ne))
        for i in range(1, ne + 1):
            rhs = forcing_domega(sysm, omega, phases, 0.0, i)
            if i == 1:
                rhs = rhs - D @ u - 2.0 * w1 * M @ a
            Aw[:, i - 1] = _solve(Mw, rhs)
    iters = np.zeros(steps, dtype=np.int64)
    qh = [q.copy()] if history else None
    for k in range(steps):
        phi_next = (k + 1) * h
        e1 = forcing(sysm, omega, phases, phi_next, phi0)
        b = e1 + Mw @ (c0 * q + c1 * u + a) + w1 * D @ (c2 * q + u)
        qn = q + h * u + 0.5 * h * h * a
        prev = math.inf
        ok = False
        for it in range(maxit):
            r = S @ qn + internal_force(sysm, qn) - b
            T = S + tangent(sysm, qn)
            dq = _solve(T, r)
            qn = qn - dq
            nd = float(np.max(np.abs(dq)))
            scale = max(float(np.max(np.abs(qn))), q_scale)
            iters[k] = it + 1
            if nd <= tol * scale or (nd <= 1e3 * tol * scale and nd > 0.5 * prev):
                ok = True
                break
            prev = nd
        if not ok:
            raise StepNewtonError(f"step Newton did not converge at step {k}")
        un = c2 * (qn - q) - u
        an = c0 * (qn - q) - c1 * u - a
        if sens or omega_sens:
            T = S + tangent(sysm, qn)
        if sens:
            rhs = Mw @ (c0 * Q + c1 * U + A) + w1 * D @ (c2 * Q + U)
            Qn = _solve(T, rhs)
            Un = c2 * (Qn - Q) - U
            An = c0 * (Qn - Q) - c1 * U - A
            Q, U, A = Qn, Un, An
        if omega_sens:
            rhs = Mw @ (c0 * Qw + c1 * Uw + Aw) + w1 * D @ (c2 * Qw + Uw)
            for i in range(1, ne + 1):
                col = forcing_domega(sysm, omega, phases, phi_next, i)
                if i == 1:
                    dS = 2.0 * w1 * c0 * M + c2 * D
                    col = (col - dS @ qn + 2.0 * w1 * M @ (c0 * q + c1 * u + a)
                           + D @ (c2 * q + u))
                rhs[:, i - 1] += col
            Qwn = _solve(T, rhs)
            Uwn = c2 * (Qwn - Qw) - Uw
            Awn = c0 * (Qwn - Qw) - c1 * Uw - Aw
            Qw, Uw, Aw = Qwn, Uwn, Awn
        q, u, a = qn, un, an
        if history:
            qh.append(q.copy())
    out = {"zT": np.concatenate([q, u]), "iters": iters, "aT": a}
    if sens:
        out["Phi"] = np.vstack([Q, U])
    if omega_sens:
        out["dz_domega"] = np.vstack([Qw, Uw])
    if history:
        out["q_hist"] = np.array(qh)
    return out


def integrate_general(sysm, omega, S1: int, phases, z0, sens: bool = False, omega_sens: bool = False,
                      tol: float = 1e-12, maxit: int = 30, q_scale: float = 0.0, history: bool = False,
                      beta: float = 0.25, gamma: float = 0.5, steps: int = None, phi0: float = 0.0):
    """The same trajectory with the general Newmark rule (the paper's future-work item 3;
    App. E is its case beta = 1/4, gamma = 1/2).  Newmark's two relations, in phi_1:
        q_{k+1} = q_k + h u_k + h^2 ((1/2 - beta) a_k + beta a_{k+1}),
        u_{k+1} = u_k + h ((1 - gamma) a_k + gamma a_{k+1}),
    so with p_k = q_k + h u_k + h^2 (1/2 - beta) a_k and v_k = u_k + h (1 - gamma) a_k,
        a_{k+1} = (q_{k+1} - p_k) / (beta h^2),  u_{k+1} = v_k + gamma h a_{k+1},
    and the equation of motion at phi_{k+1} is solved for q_{k+1} by full-tangent Newton with
    the tangent T = w1^2 M / (beta h^2) + w1 D gamma / (beta h) + K + K_t(q_{k+1}).  The
    sensitivities differentiate these relations at the converged step: T dq_{k+1} =
    w1^2 M dp / (beta h^2) + w1 D (gamma / (beta h) dp - dv), and the same for d/d omega with
    the explicit terms -(2 w1 M a_{k+1} + D u_{k+1}) (omega_1 only) and d e / d omega."""
    M, D, K = sysm.M, sysm.D, sysm.K
    n = sysm.n
    steps = S1 if steps is None else steps
    omega = np.asarray(omega, dtype=float)
    w1 = omega[0]
    h = 2.0 * math.pi / S1
    ca = 1.0 / (beta * h * h)          # d a_{k+1} / d q_{k+1}
    cu = gamma / (beta * h)            # d u_{k+1} / d q_{k+1}
    Mw = w1 ** 2 * M
    S = ca * Mw + cu * w1 * D + K
    q = np.array(z0[:n], dtype=float)
    u = np.array(z0[n:], dtype=float)
    vel = has_velocity(sysm)

    def forces(qq, uu):
        """f_nl, K_t and C_t at the state (q, u), qdot = w1 u."""
        qd = w1 * uu if vel else None
        Kt, Ct = tangents(sysm, qq, qd)
        return internal_force(sysm, qq, qd), Kt, Ct

    f0, Kt0, Ct0 = forces(q, u)
    a = _solve(Mw, forcing(sysm, omega, phases, 0.0, phi0) - w1 * D @ u - K @ q - f0)
    if sens:
        Q = np.hstack([np.eye(n), np.zeros((n, n))])
        U = np.hstack([np.zeros((n, n)), np.eye(n)])
        A = -_solve(Mw, np.hstack([K + Kt0, w1 * (D + Ct0)]))
    ne = sysm.e
    if omega_sens:
        Qw = np.zeros((n, ne))
        Uw = np.zeros((n, ne))
        Aw = np.zeros((n, ne))
        for i in range(1, ne + 1):
            rhs = forcing_domega(sysm, omega, phases, 0.0, i)
            if i == 1:
                rhs = rhs - (D + Ct0) @ u - 2.0 * w1 * M @ a
            Aw[:, i - 1] = _solve(Mw, rhs)
    iters = np.zeros(steps, dtype=np.int64)
    qh = [q.copy()] if history else None

    def accel_vel(qn, p, v):
        an = (qn - p) / (beta * h * h)
        return an, v + gamma * h * an

    for k in range(steps):
        phi_next = (k + 1) * h
        e1 = forcing(sysm, omega, phases, phi_next, phi0)
        p = q + h * u + h * h * (0.5 - beta) * a
        v = u + h * (1.0 - gamma) * a
        qn = q + h * u + 0.5 * h * h * a
        prev = math.inf
        ok = False
        for it in range(maxit):
            an, un = accel_vel(qn, p, v)
            fq, Kt, Ct = forces(qn, un)
            r = Mw @ an + w1 * D @ un + K @ qn + fq - e1
            dq = _solve(S + Kt + w1 * cu * Ct, r)
            qn = qn - dq
            nd = float(np.max(np.abs(dq)))
            scale = max(float(np.max(np.abs(qn))), q_scale)
            iters[k] = it + 1
            if nd <= tol * scale or (nd <= 1e3 * tol * scale and nd > 0.5 * prev):
                ok = True
                break
            prev = nd
        if not ok:
            raise StepNewtonError(f"step Newton did not converge at step {k}")
        an, un = accel_vel(qn, p, v)
        if sens or omega_sens:
            _, Kt, Ct = forces(qn, un)
            T = S + Kt + w1 * cu * Ct
            Deff = D + Ct  # the velocity-dependent forces linearise into a state-dependent damping
        if sens:
            dP = Q + h * U + h * h * (0.5 - beta) * A
            dV = U + h * (1.0 - gamma) * A
            Qn = _solve(T, ca * Mw @ dP + w1 * Deff @ (cu * dP - dV))
            An = (Qn - dP) / (beta * h * h)
            Un = dV + gamma * h * An
            Q, U, A = Qn, Un, An
        if omega_sens:
            dP = Qw + h * Uw + h * h * (0.5 - beta) * Aw
            dV = Uw + h * (1.0 - gamma) * Aw
            rhs = ca * Mw @ dP + w1 * Deff @ (cu * dP - dV)
            for i in range(1, ne + 1):
                col = forcing_domega(sysm, omega, phases, phi_next, i)
                if i == 1:
                    col = col - 2.0 * w1 * M @ an - Deff @ un
                rhs[:, i - 1] += col
            Qwn = _solve(T, rhs)
            Awn = (Qwn - dP) / (beta * h * h)
            Uwn = dV + gamma * h * Awn
            Qw, Uw, Aw = Qwn, Uwn, Awn
        q, u, a = qn, un, an
        if history:
            qh.append(q.copy())
    out = {"zT": np.concatenate([q, u]), "iters": iters, "aT": a}
    if sens:
        out["Phi"] = np.vstack([Q, U])
    if omega_sens:
        out["dz_domega"] = np.vstack([Qw, Uw])
    if history:
        out["q_hist"] = np.array(qh)
    return out

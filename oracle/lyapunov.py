"""Lyapunov exponents from the FSE-Shooting by-product (oracle; test infrastructure only).

App. F: the one-period transition matrix of the trajectory that starts on the
initial section at phi~ is Psi(phi~) (Eq. F3), obtained from the sensitivity
Phi_s = d[q;u](2pi)/d[q;u](0) by the change of variables qdot = omega_1 u.  It
is a quasi-periodic function of phi~, interpolated by trigonometric polynomials
on the torus grid; step i of the discrete Gram-Schmidt (Eq. F2) uses
Psi(2 pi (i-1) rho) with the interval Delta t = T_1 = 2 pi / omega_1.

Readings: the interpolation basis is the torus basis
H(k~, phi~) with coefficients Gamma^-1 Psi_s (the "(d-1)-dimensional FFT");
the Gram-Schmidt is a Householder QR with a positive diagonal; the exponents
are returned in QR column order and sorted.

Pins (tests/test_oracle_lyapunov.py): sum of exponents = mean log|det Psi_i|
(exact for any system), linear systems (constant Psi): exponents = log|mu|/T_1
of the eigenvalues of the trapezoidal one-period map, and the continuous-time
limit sum = -tr(M^-1 D) for a resolved 2-DOF system.
"""
from __future__ import annotations

import math

import numpy as np

from . import torus as tor


def transition_samples(Phi: np.ndarray, omega1: float) -> np.ndarray:
    """Eq. (F3): Psi_s = diag(I, w1 I) Phi_s diag(I, I / w1) for every sample s."""
    n2 = Phi.shape[1]
    n = n2 // 2
    sc = np.concatenate([np.ones(n), np.full(n, omega1)])
    return Phi * sc[None, :, None] / sc[None, None, :]


def exponents(Phi: np.ndarray, omega, tables, N_Ly: int = 1000, Q0=None):
    """Returns (sigma in QR order, sigma sorted descending, log|R_hh| sums).

    Q0 is the initial orthonormal basis of the Gram-Schmidt sweep (identity,
    i.e. Psi(t_0, t_0) = I, when None).  A generic basis avoids the long
    transient of a start plane that is nearly orthogonal to a dominant
    invariant subspace (decoupled systems)."""
    omega = np.asarray(omega, dtype=float)
    w1 = omega[0]
    rho = omega[1:] / w1
    Psi = transition_samples(Phi, w1)
    # trigonometric-polynomial coefficients of Psi(phi~): Gamma^-1 over s
    Psihat = np.einsum("ls,sij->lij", tables.Gi, Psi)
    n2 = Phi.shape[1]
    Qm = np.eye(n2) if Q0 is None else np.array(Q0, dtype=float)
    acc = np.zeros(n2)
    for i in range(1, N_Ly + 1):
        phi = 2.0 * math.pi * (i - 1) * rho
        H = tor.trig_row(tables.table, phi)
        Psi_i = np.einsum("l,lij->ij", H, Psihat)
        Y = Psi_i @ Qm
        Qm, Rm = np.linalg.qr(Y)
        sgn = np.sign(np.diag(Rm))
        sgn[sgn == 0] = 1.0
        Qm = Qm * sgn[None, :]
        Rm = Rm * sgn[:, None]
        acc += np.log(np.abs(np.diag(Rm)))
    T1 = 2.0 * math.pi / w1
    sig = acc / (N_Ly * T1)
    return sig, np.sort(sig)[::-1], acc


def interpolated_transition(Phi, omega, tables, phi):
    """Psi(phi~) at an arbitrary point (used by tests)."""
    omega = np.asarray(omega, dtype=float)
    Psi = transition_samples(Phi, omega[0])
    Psihat = np.einsum("ls,sij->lij", tables.Gi, Psi)
    return np.einsum("l,lij->ij", tor.trig_row(tables.table, phi), Psihat)

"""Closed forms shared by the oracle pins."""
import math

import numpy as np

from fse_inputs.systems import place_harmonics


def discrete_linear_torus(s, omega, S1, table, U):
    """Closed-form steady state of the *discrete* Newmark map of a linear system.

    For forcing F_i cos(lambda_i phi_1 + psi_i) the trapezoidal recurrence has the
    particular solution q = Re[Qh e^{i(lambda phi_1 + psi)}] with frequency
    distortion lambda~ = (2/h) tan(lambda h / 2):  u = Re[i lambda~ Qh ...],
    a = Re[-lambda~^2 Qh ...], (K - w1^2 lambda~^2 M + i w1 lambda~ D) Qh = F_i.
    """
    h = 2 * math.pi / S1
    w1 = omega[0]
    harms = []
    for i in range(s.e):
        lam = omega[i] / w1
        lt = (2 / h) * math.tan(lam * h / 2)
        A = s.K - w1 ** 2 * lt ** 2 * s.M + 1j * w1 * lt * s.D
        Qh = np.linalg.solve(A, s.F[i].astype(complex))
        k = (0,) if i == 0 else tuple(1 if j == i - 1 else 0 for j in range(len(omega) - 1))
        harms.append((k, np.concatenate([Qh, 1j * lt * Qh])))
    return place_harmonics(table, harms, s.n, U)


def discrete_linear_sections(s, omega, S1, table, U, M):
    """Closed-form steady state of the discrete (trapezoidal) Newmark map of a linear system
    on the sections phi_1 = 2 pi m / M: the harmonic of frequency 1 at phase 2 pi m / M, the
    others in the section's own phases (distorted frequency (2/h) tan(lambda h / 2))."""
    h = 2 * math.pi / S1
    w1 = omega[0]
    out = []
    for m in range(M):
        harms = []
        for i in range(s.e):
            lam = omega[i] / w1
            lt = (2 / h) * math.tan(lam * h / 2)
            Qh = np.linalg.solve(s.K - w1 ** 2 * lt ** 2 * s.M + 1j * w1 * lt * s.D, s.F[i].astype(complex))
            if i == 0:
                Qh = Qh * np.exp(2j * math.pi * m / M)
            k = (0,) if i == 0 else tuple(1 if j == i - 1 else 0 for j in range(len(omega) - 1))
            harms.append((k, np.concatenate([Qh, 1j * lt * Qh])))
        out.append(place_harmonics(table, harms, s.n, U))
    return np.array(out)

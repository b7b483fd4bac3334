"""Pins of the oracle's velocity-dependent forces f_nl(q, qdot) (Eq. 1; the paper's outlook)."""
import math

import numpy as np
import pytest

from _velocity_systems import mixed_system, van_der_pol
from fse_inputs import Torus
from fse_inputs.systems import place_harmonics
from oracle import lyapunov as oly
from oracle import newmark
from oracle import shooting as osh


@pytest.mark.parametrize("beta,gamma", [(0.25, 0.5), (0.3025, 0.6)])
def test_sensitivities_match_finite_differences(beta, gamma):
    s = mixed_system()
    assert newmark.has_velocity(s)
    omega = np.array([1.1, 1.1 * 1.618])
    phases = np.array([0.9])
    z0 = 0.3 * np.random.default_rng(7).normal(size=6)
    out = newmark.integrate(s, omega, 48, phases, z0, sens=True, omega_sens=True, beta=beta, gamma=gamma)
    h = 1e-6
    J = np.zeros((6, 6))
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        zp = newmark.integrate(s, omega, 48, phases, z0 + e, beta=beta, gamma=gamma)["zT"]
        zm = newmark.integrate(s, omega, 48, phases, z0 - e, beta=beta, gamma=gamma)["zT"]
        J[:, j] = (zp - zm) / (2 * h)
    assert np.allclose(out["Phi"], J, rtol=1e-6, atol=1e-7)
    for i in range(2):
        e = np.zeros(2)
        e[i] = h
        zp = newmark.integrate(s, omega + e, 48, phases, z0, beta=beta, gamma=gamma)["zT"]
        zm = newmark.integrate(s, omega - e, 48, phases, z0, beta=beta, gamma=gamma)["zT"]
        assert np.allclose(out["dz_domega"][:, i], (zp - zm) / (2 * h), rtol=1e-6, atol=1e-7)


def test_tangents_are_the_derivatives_of_the_force():
    s = mixed_system()
    rng = np.random.default_rng(3)
    q, qd = rng.normal(size=3), rng.normal(size=3)
    Kt, Ct = newmark.tangents(s, q, qd)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fk = (newmark.internal_force(s, q + e, qd) - newmark.internal_force(s, q - e, qd)) / (2 * h)
        fc = (newmark.internal_force(s, q, qd + e) - newmark.internal_force(s, q, qd - e)) / (2 * h)
        assert np.allclose(Kt[:, j], fk, rtol=1e-7, atol=1e-9)
        assert np.allclose(Ct[:, j], fc, rtol=1e-7, atol=1e-9)
    assert np.allclose(Kt, Kt.T) and np.allclose(Ct, Ct.T)


def vdp_case(mu=0.2):
    s = van_der_pol(mu=mu)
    w1 = 2.3
    tr = Torus(d=2, e=1, K=[np.arange(1, 8)], S=[16], S1=128)
    tb = osh.TorusTables(tr)
    A = 0.5 / (1 - w1 ** 2)
    Z0 = place_harmonics(tb.table, [((0,), np.array([A, 0.0], complex)), ((1,), np.array([2.0, 2j / w1]))],
                         1, tb.U)
    return s, tr, tb, np.array([w1, 1.0]), Z0


def test_forced_van_der_pol_torus():
    """Self-excited oscillator forced off resonance (d = 2, e = 1, omega_2 unknown): the
    limit-cycle frequency is 1 - mu^2/16 and its amplitude 2 to the order of the classical
    averaging result; the torus has one zero Lyapunov exponent (the free phase of the
    self-excited oscillation) and one near -mu (the contraction onto the limit cycle)."""
    mu = 0.2
    s, tr, tb, om, Z0 = vdp_case(mu)
    Z, omf, hist = osh.solve(s, tr, om, Z0, tol_R=1e-10, max_newton=25, tables=tb)
    assert hist[-1] < 1e-10
    assert abs(omf[1] - (1 - mu ** 2 / 16)) < 2e-4
    l = [tuple(r) for r in tb.table].index((1,))
    assert abs(math.hypot(Z[0, 2 * l + 1], Z[0, 2 * l + 2]) - 2.0) < 0.02
    res = osh.evaluate(s, tr, omf, Z, sens=True, tables=tb)
    sig = oly.exponents(res["Phi"], omf, tb, N_Ly=400)[1]
    assert abs(sig[0]) < 2e-3
    assert abs(sig[1] + mu) < 0.05 * mu

"""Pins of the oracle's nonsmooth forces: unilateral penalty contacts, piecewise linear in q
(the paper's third recommendation, extension to nonsmooth systems)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from _velocity_systems import impact_oscillator, with_contacts
from fse_inputs import Torus, tiny_system
from oracle import lyapunov as oly
from oracle import newmark
from oracle import shooting as osh


def stepped_by_cases(c, kc, gap, F, w, S1, z0, two_sided):
    """One period of the average-acceleration rule for the 1-DOF impact oscillator, each step
    equation S q + f_c(q) = b solved by its case split (f_c is monotone and piecewise linear)."""
    h = 2 * math.pi / S1
    c0, c1, c2 = 4 / h ** 2, 4 / h, 2 / h
    S = w * w * c0 + w * c2 * c + 1.0

    def fc(q):
        return kc * max(q - gap, 0.0) - (kc * max(-q - gap, 0.0) if two_sided else 0.0)

    q, u = z0
    a = (F - w * c * u - q - fc(q)) / (w * w)
    for k in range(S1):
        b = F * math.cos((k + 1) * h) + w * w * (c0 * q + c1 * u + a) + w * c * (c2 * q + u)
        if b > S * gap:
            qn = (b + kc * gap) / (S + kc)
        elif two_sided and b < -S * gap:
            qn = (b - kc * gap) / (S + kc)
        else:
            qn = b / S
        un = c2 * (qn - q) - u
        a = c0 * (qn - q) - c1 * u - a
        q, u = qn, un
    return np.array([q, u])


@pytest.mark.parametrize("two_sided", [False, True])
@pytest.mark.parametrize("general", [False, True])
def test_step_equation_against_case_split(two_sided, general):
    c, kc, gap, F, w = 0.2, 4.0, 0.3, 0.6, 1.3
    s = impact_oscillator(c, kc, gap, F, two_sided)
    for z0 in ([0.0, 0.0], [0.5, -0.4], [-0.7, 0.2]):
        ref = stepped_by_cases(c, kc, gap, F, w, 96, z0, two_sided)
        out = newmark.integrate(s, np.array([w]), 96, np.zeros(0), np.array(z0), general=general)
        assert np.allclose(out["zT"], ref, rtol=1e-12, atol=1e-13)
        free = newmark.integrate(impact_oscillator(c, 0.0, gap, F, two_sided), np.array([w]), 96,
                                 np.zeros(0), np.array(z0))["zT"]
        assert np.linalg.norm(free - ref) > 1e-3          # the stops were hit


def test_open_contacts_change_nothing():
    s0 = tiny_system(n=3, seed=2, cubic=1.0, quad=0.3, e=2)
    s = with_contacts(s0, [0, 2], [1, -1], [50.0, 50.0], [7.0, 7.0])
    om = np.array([1.1, 1.1 * 1.618])
    z0 = 0.3 * np.random.default_rng(1).normal(size=6)
    a = newmark.integrate(s, om, 48, np.array([0.4]), z0, sens=True)
    b = newmark.integrate(s0, om, 48, np.array([0.4]), z0, sens=True)
    assert np.array_equal(a["zT"], b["zT"]) and np.array_equal(a["Phi"], b["Phi"])


@pytest.mark.parametrize("beta,gamma", [(0.25, 0.5), (0.3025, 0.6)])
def test_sensitivities_match_finite_differences(beta, gamma):
    s0 = tiny_system(n=3, seed=2, cubic=1.0, quad=0.3, e=2)
    s = with_contacts(s0, [0, 2, 1], [1, -1, 1], [0.05, 0.02, 0.0], [5.0, 3.0, 2.0])
    om = np.array([1.1, 1.1 * 1.618])
    ph = np.array([0.9])
    z0 = 0.3 * np.random.default_rng(7).normal(size=6)
    out = newmark.integrate(s, om, 48, ph, z0, sens=True, omega_sens=True, beta=beta, gamma=gamma)
    free = newmark.integrate(s0, om, 48, ph, z0, beta=beta, gamma=gamma)["zT"]
    assert np.linalg.norm(free - out["zT"]) > 1e-3
    h = 1e-5   # every closed or open contact stays > 2e-4 from its gap along this trajectory
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        zp = newmark.integrate(s, om, 48, ph, z0 + e, beta=beta, gamma=gamma)["zT"]
        zm = newmark.integrate(s, om, 48, ph, z0 - e, beta=beta, gamma=gamma)["zT"]
        assert np.allclose(out["Phi"][:, j], (zp - zm) / (2 * h), rtol=1e-6, atol=1e-7)
    for i in range(2):
        e = np.zeros(2)
        e[i] = h
        zp = newmark.integrate(s, om + e, 48, ph, z0, beta=beta, gamma=gamma)["zT"]
        zm = newmark.integrate(s, om - e, 48, ph, z0, beta=beta, gamma=gamma)["zT"]
        assert np.allclose(out["dz_domega"][:, i], (zp - zm) / (2 * h), rtol=1e-6, atol=1e-7)


def test_impact_orbit_converges_at_second_order():
    """Forced impact oscillator (d = 1): the shooting orbit's defect against the exact flow
    (integrated piecewise, restarted at every contact event) falls by 4 when S_1 doubles."""
    c, kc, gap, F = 0.2, 4.0, 0.3, 0.6
    s = impact_oscillator(c, kc, gap, F)
    w = 1.3

    def rhs(t, y):
        return [y[1], F * math.cos(w * t) - c * y[1] - y[0] - kc * max(y[0] - gap, 0.0)]

    def hit(t, y):
        return y[0] - gap

    def flow(z):
        t, y, T = 0.0, [z[0], z[1] * w], 2 * math.pi / w
        while t < T:
            sol = solve_ivp(rhs, [t, T], y, method="DOP853", rtol=1e-13, atol=1e-15, events=hit)
            t, y = sol.t[-1], sol.y[:, -1]
            if sol.status == 1:          # stepped to the event: restart just past it
                nxt = solve_ivp(rhs, [t, min(t + 1e-9, T)], y, method="DOP853", rtol=1e-13, atol=1e-15)
                t, y = nxt.t[-1], nxt.y[:, -1]
        return np.array([y[0], y[1] / w])

    defects = []
    for S1 in (256, 512):
        tr = Torus(d=1, e=1, K=[], S=[], S1=S1)
        tb = osh.TorusTables(tr)
        Z, _, hist = osh.solve(s, tr, np.array([w]), np.zeros((2, 1)), tol_R=1e-12, tables=tb)
        assert hist[-1] < 1e-12
        qh = newmark.integrate(s, np.array([w]), S1, np.zeros(0), Z[:, 0], history=True)["q_hist"]
        assert np.max(qh) > gap + 0.05            # the orbit strikes the stop
        defects.append(np.abs(flow(Z[:, 0]) - Z[:, 0]).max())
    assert 3.0 < defects[0] / defects[1] < 5.0


def test_impact_orbit_is_the_attractor_and_symmetric():
    """The shooting orbit is where a long transient from rest ends (damped system), its
    Lyapunov exponents are negative, and two symmetric stops make it half-wave symmetric:
    half a period of forcing maps z* to -z*."""
    c, kc, gap, F, w = 0.2, 4.0, 0.3, 0.6, 1.3
    for two in (False, True):
        s = impact_oscillator(c, kc, gap, F, two)
        tr = Torus(d=1, e=1, K=[], S=[], S1=128)
        tb = osh.TorusTables(tr)
        Z, _, hist = osh.solve(s, tr, np.array([w]), np.zeros((2, 1)), tol_R=1e-12, tables=tb)
        assert hist[-1] < 1e-12
        z = np.zeros(2)
        for _ in range(120):
            z = newmark.integrate(s, np.array([w]), 128, np.zeros(0), z)["zT"]
        assert np.allclose(z, Z[:, 0], atol=1e-11)
        res = osh.evaluate(s, tr, np.array([w]), Z, sens=True, tables=tb)
        sig = np.linalg.eigvals(res["Phi"][0])
        assert np.max(np.abs(sig)) < 1.0
        if two:
            half = newmark.integrate(s, np.array([w]), 128, np.zeros(0), Z[:, 0], steps=64)["zT"]
            assert np.allclose(half, -Z[:, 0], atol=1e-11)

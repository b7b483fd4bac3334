"""Pins of the oracle's Newmark integrator and its sensitivities (App. E)."""
import math

import numpy as np
import pytest

from fse_inputs import linear_oscillator, tiny_system
from oracle import newmark


@pytest.mark.parametrize("Omega,S1", [(2.3, 64), (0.4, 16), (7.0, 32)])
def test_undamped_oscillator_closed_form(Omega, S1):
    """Average acceleration = trapezoidal rule: x_k = x0 cos(k th) + v0/W sin(k th),
    th = 2 atan(W h / 2), unit amplification (standard result for this scheme)."""
    sysm = linear_oscillator(Omega=Omega)
    w1 = 1.0
    x0, v0 = 0.7, -0.3
    out = newmark.integrate(sysm, [w1], S1, np.zeros(0), np.array([x0, v0]))
    h = 2 * math.pi / S1
    th = 2 * math.atan(Omega * h / 2)
    xk = x0 * math.cos(S1 * th) + v0 / Omega * math.sin(S1 * th)
    vk = -x0 * Omega * math.sin(S1 * th) + v0 * math.cos(S1 * th)
    assert abs(out["zT"][0] - xk) < 1e-12
    assert abs(out["zT"][1] - vk) < 1e-12
    amp0 = x0 ** 2 + (v0 / Omega) ** 2
    amp1 = out["zT"][0] ** 2 + (out["zT"][1] / Omega) ** 2
    assert abs(amp1 - amp0) < 1e-13


def test_period_elongation_formula():
    """Relative period error (W h / 2) / atan(W h / 2) - 1 ~ (W h)^2 / 12."""
    Omega, S1 = 1.0, 40
    h = 2 * math.pi / S1
    th = 2 * math.atan(Omega * h / 2)
    sysm = linear_oscillator(Omega=Omega)
    out = newmark.integrate(sysm, [1.0], S1, np.zeros(0), np.array([1.0, 0.0]))
    # after one physical period 2 pi the numerical phase is S1 * th < 2 pi
    assert abs(out["zT"][0] - math.cos(S1 * th)) < 1e-13
    ratio = (Omega * h / 2) / math.atan(Omega * h / 2)
    assert abs((ratio - 1) - (Omega * h) ** 2 / 12) < 0.1 * (Omega * h) ** 2 / 12


def test_undamped_mdof_energy_conserved():
    """Linear undamped MDOF: the trapezoidal map conserves u^T (w^2 M) u + q^T K q exactly."""
    s = tiny_system(n=4, seed=2, nonlinear=False, zeta=0.0)
    s.D[:] = 0.0
    s.F[:] = 0.0
    w1 = 1.7
    rng = np.random.default_rng(0)
    z0 = rng.normal(size=8)
    out = newmark.integrate(s, [w1, 2.0], 50, np.zeros(1), z0)
    q0, u0 = z0[:4], z0[4:]
    q1, u1 = out["zT"][:4], out["zT"][4:]
    E0 = u0 @ (w1 ** 2 * s.M) @ u0 + q0 @ s.K @ q0
    E1 = u1 @ (w1 ** 2 * s.M) @ u1 + q1 @ s.K @ q1
    assert abs(E1 - E0) < 1e-12 * E0


def test_consistent_initial_acceleration():
    """a_0 satisfies the trajectory equation (E2) at phi_1 = 0; with q0 = u0 = 0 and
    no forcing every step stays at rest."""
    s = tiny_system(n=3, seed=3)
    s.F[:] = 0.0
    out = newmark.integrate(s, [1.0, 1.5], 20, np.zeros(1), np.zeros(6))
    assert np.all(out["zT"] == 0.0)


def _fd_sens(s, omega, S1, phases, z0, h=1e-6):
    n2 = len(z0)
    J = np.zeros((n2, n2))
    for j in range(n2):
        e = np.zeros(n2)
        e[j] = h
        zp = newmark.integrate(s, omega, S1, phases, z0 + e)["zT"]
        zm = newmark.integrate(s, omega, S1, phases, z0 - e)["zT"]
        J[:, j] = (zp - zm) / (2 * h)
    return J


@pytest.mark.parametrize("seed", [1, 7])
def test_sensitivity_matches_finite_differences(seed):
    s = tiny_system(n=3, seed=seed, cubic=2.0, quad=0.5)
    omega = np.array([1.1, 1.1 * 1.618])
    phases = np.array([0.9])
    rng = np.random.default_rng(seed)
    z0 = 0.3 * rng.normal(size=6)
    out = newmark.integrate(s, omega, 48, phases, z0, sens=True)
    fd = _fd_sens(s, omega, 48, phases, z0)
    assert np.allclose(out["Phi"], fd, rtol=1e-6, atol=1e-7)


def test_linear_sensitivity_is_power_of_one_step_map():
    """Linear system: Phi = G^S1 with G the one-step map of [q; u] (brute force)."""
    s = tiny_system(n=2, seed=4, nonlinear=False)
    omega = np.array([0.9, 1.3])
    S1 = 16
    out = newmark.integrate(s, omega, S1, np.zeros(1), np.zeros(4), sens=True)
    # one step of size 2 pi / S1 == one step of S1' = 1 with omega' = S1 omega (same
    # physical step); then u' = dq/dphi' = u / S1, so conjugate by C = diag(1, S1).
    om2 = omega * S1
    G = np.zeros((4, 4))
    base = newmark.integrate(s, om2, 1, np.zeros(1), np.zeros(4))["zT"]
    for j in range(4):
        e = np.zeros(4)
        e[j] = 1.0
        G[:, j] = newmark.integrate(s, om2, 1, np.zeros(1), e)["zT"] - base
    C = np.diag([1, 1, S1, S1]).astype(float)
    Gs = C @ G @ np.linalg.inv(C)
    assert np.allclose(out["Phi"], np.linalg.matrix_power(Gs, S1), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("i", [1, 2])
def test_omega_sensitivity_matches_finite_differences(i):
    s = tiny_system(n=3, seed=5, cubic=1.0, quad=0.3)
    omega = np.array([1.2, 1.2 * 1.4142])
    phases = np.array([2.1])
    rng = np.random.default_rng(1)
    z0 = 0.2 * rng.normal(size=6)
    out = newmark.integrate(s, omega, 40, phases, z0, omega_sens=True)
    h = 1e-6
    e = np.zeros(2)
    e[i - 1] = h
    zp = newmark.integrate(s, omega + e, 40, phases, z0)["zT"]
    zm = newmark.integrate(s, omega - e, 40, phases, z0)["zT"]
    assert np.allclose(out["dz_domega"][:, i - 1], (zp - zm) / (2 * h), rtol=1e-6, atol=1e-7)


# ---------------------------------------------------------------- general Newmark (beta, gamma)
GENERAL = [(1.0 / 6.0, 0.5), (0.3, 0.5), (0.3025, 0.6), (0.4, 0.7)]


@pytest.mark.parametrize("sens", [False, True])
def test_general_rule_at_quarter_half_is_the_average_acceleration_rule(sens):
    """The general branch, forced at (1/4, 1/2), reproduces App. E's branch (states,
    sensitivities and omega-derivatives) on a nonlinear two-frequency system."""
    s = tiny_system(n=3, seed=5, cubic=1.0, quad=0.3)
    omega = np.array([1.2, 1.2 * 1.4142])
    phases = np.array([2.1])
    z0 = 0.2 * np.random.default_rng(1).normal(size=6)
    a = newmark.integrate(s, omega, 40, phases, z0, sens=sens, omega_sens=sens)
    b = newmark.integrate(s, omega, 40, phases, z0, sens=sens, omega_sens=sens, general=True)
    assert np.allclose(a["zT"], b["zT"], rtol=1e-12, atol=1e-14)
    if sens:
        assert np.allclose(a["Phi"], b["Phi"], rtol=1e-11, atol=1e-13)
        assert np.allclose(a["dz_domega"], b["dz_domega"], rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("beta,gamma", GENERAL)
def test_general_rule_obeys_the_three_term_recurrence(beta, gamma):
    """Undamped oscillator q'' + W^2 q = 0: eliminating u and a from Newmark's relations gives
    the textbook three-term recurrence (1 + b x) q_{k+1} - (2 - (1/2 - 2b + g) x) q_k
    + (1 + (1/2 + b - g) x) q_{k-1} = 0, x = (W h)^2.  The oracle's displacements are
    c1 l1^k + c2 l2^k with l1, l2 the roots of its characteristic polynomial."""
    Omega, S1 = 1.7, 48
    sysm = linear_oscillator(Omega=Omega)
    out = newmark.integrate(sysm, [1.0], S1, np.zeros(0), np.array([0.6, -0.4]), beta=beta, gamma=gamma,
                            history=True)
    qk = out["q_hist"][:, 0]
    h = 2 * math.pi / S1
    x = (Omega * h) ** 2
    lam = np.roots([1 + beta * x, -(2 - (0.5 - 2 * beta + gamma) * x), 1 + (0.5 + beta - gamma) * x])
    V = np.array([[1.0, 1.0], lam]).astype(complex)
    c = np.linalg.solve(V, qk[:2].astype(complex))
    model = (c[None, :] * lam[None, :] ** np.arange(len(qk))[:, None]).sum(axis=1)
    assert np.abs(model.imag).max() < 1e-12
    assert np.abs(model.real - qk).max() < 1e-12 * np.abs(qk).max()
    # no numerical damping at gamma = 1/2, decay above it (|l|^2 = product of the roots)
    rho2 = (1 + (0.5 + beta - gamma) * x) / (1 + beta * x)
    assert abs(np.abs(lam).max() ** 2 - rho2) < 1e-14 if gamma > 0.5 else abs(rho2 - 1.0) < 1e-15


@pytest.mark.parametrize("beta,gamma,order", [(0.3, 0.5, 2), (1.0 / 6.0, 0.5, 2), (0.3025, 0.6, 1)])
def test_general_rule_order_of_accuracy(beta, gamma, order):
    """Error against the exact cos(W t) after one period halves like h^2 for gamma = 1/2 and
    like h for gamma != 1/2 (Newmark's classical accuracy result)."""
    Omega = 1.3
    sysm = linear_oscillator(Omega=Omega)
    errs = []
    for S1 in (200, 400, 800):
        out = newmark.integrate(sysm, [1.0], S1, np.zeros(0), np.array([1.0, 0.0]), beta=beta, gamma=gamma)
        errs.append(abs(out["zT"][0] - math.cos(Omega * 2 * math.pi)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.15 for r in rates), rates


@pytest.mark.parametrize("beta,gamma", [(0.3025, 0.6), (1.0 / 6.0, 0.5)])
def test_general_rule_sensitivities_match_finite_differences(beta, gamma):
    s = tiny_system(n=3, seed=7, cubic=2.0, quad=0.5)
    omega = np.array([1.1, 1.1 * 1.618])
    phases = np.array([0.9])
    z0 = 0.3 * np.random.default_rng(7).normal(size=6)
    out = newmark.integrate(s, omega, 48, phases, z0, sens=True, omega_sens=True, beta=beta, gamma=gamma)
    hh = 1e-6
    J = np.zeros((6, 6))
    for j in range(6):
        e = np.zeros(6)
        e[j] = hh
        zp = newmark.integrate(s, omega, 48, phases, z0 + e, beta=beta, gamma=gamma)["zT"]
        zm = newmark.integrate(s, omega, 48, phases, z0 - e, beta=beta, gamma=gamma)["zT"]
        J[:, j] = (zp - zm) / (2 * hh)
    assert np.allclose(out["Phi"], J, rtol=1e-6, atol=1e-7)
    for i in range(2):
        e = np.zeros(2)
        e[i] = hh
        zp = newmark.integrate(s, omega + e, 48, phases, z0, beta=beta, gamma=gamma)["zT"]
        zm = newmark.integrate(s, omega - e, 48, phases, z0, beta=beta, gamma=gamma)["zT"]
        assert np.allclose(out["dz_domega"][:, i], (zp - zm) / (2 * hh), rtol=1e-6, atol=1e-7)


def test_sensitivity_column_subset_equals_the_full_columns():
    """sens_cols propagates chosen columns of Phi by the same recursion: they equal those
    columns of the full Phi (which central differences pin), in any order and with repeats."""
    from fse_inputs import tiny_system
    s = tiny_system(n=4, seed=5, cubic=1.0, quad=0.3, e=2)
    om = np.array([0.9, 0.9 * 1.618])
    z0 = 0.3 * np.random.default_rng(9).normal(size=8)
    full = newmark.integrate(s, om, 40, np.array([0.7]), z0, sens=True)["Phi"]
    cols = [7, 0, 3, 3, 5]
    sub = newmark.integrate(s, om, 40, np.array([0.7]), z0, sens=True, sens_cols=cols)["Phi"]
    assert sub.shape == (8, len(cols))
    assert np.allclose(sub, full[:, cols], rtol=1e-13, atol=1e-14)

"""Pins of the oracle's shooting residual, Jacobian and Newton step (Sec. 3, Eqs. 20-24)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from fse_inputs import Torus, tiny_system
from fse_inputs.systems import place_harmonics
from oracle import shooting
from oracle import torus as tor

from _closed_forms import discrete_linear_torus as _discrete_linear_torus

GOLDEN = (1 + 5 ** 0.5) / 2


@pytest.mark.parametrize("d", [2, 3])
def test_linear_torus_closed_form_and_one_newton_step(d):
    s = tiny_system(n=3, seed=2, nonlinear=False, e=d)
    if d == 3:
        s.F[2, 1] = 0.8
    om = np.array([1.3, 1.3 * GOLDEN, 1.3 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=d, K=[np.arange(1, 4)] * (d - 1), S=[8] * (d - 1), S1=64)
    tb = shooting.TorusTables(tr)
    Zs = _discrete_linear_torus(s, om, tr.S1, tb.table, tb.U)
    res = shooting.evaluate(s, tr, om, Zs, tables=tb)
    assert np.linalg.norm(res["R"]) < 1e-12 * np.linalg.norm(Zs)
    # Newton is exact for a linear problem: one step from zero reaches the torus
    Z1, _, r0 = shooting.newton_step(s, tr, om, np.zeros_like(Zs), tables=tb)
    assert r0 > 1e-3
    assert np.allclose(Z1, Zs, atol=1e-12 * np.abs(Zs).max())


def test_discrete_vs_continuous_linear_torus():
    """The discrete torus differs from the continuous response by the frequency
    distortion tan(x)/x - 1 ~ (lambda h)^2 / 12 (second-order accuracy)."""
    s = tiny_system(n=2, seed=3, nonlinear=False, e=2)
    om = np.array([0.8, 0.8 * GOLDEN])
    errs = []
    for S1 in (64, 128):
        tr = Torus(d=2, e=2, K=[np.arange(1, 3)], S=[8], S1=S1)
        tb = shooting.TorusTables(tr)
        Zd = _discrete_linear_torus(s, om, S1, tb.table, tb.U)
        harms = []
        for i in range(2):
            lam = om[i] / om[0]
            A = s.K - om[i] ** 2 * s.M + 1j * om[i] * s.D
            Qh = np.linalg.solve(A, s.F[i].astype(complex))
            harms.append(((0,) if i == 0 else (1,), np.concatenate([Qh, 1j * lam * Qh])))
        Zc = place_harmonics(tb.table, harms, s.n, tb.U)
        errs.append(np.abs(Zd - Zc).max() / np.abs(Zc).max())
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_linear_jacobian_is_kronecker():
    """Linear system: every Phi_s is the same Phi and Eq. (22) gives Phi (x) R(rho) - I."""
    s = tiny_system(n=2, seed=5, nonlinear=False)
    om = np.array([1.1, 1.1 * GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 3)], S=[5], S1=24)
    tb = shooting.TorusTables(tr)
    Z0 = np.random.default_rng(0).normal(size=(4, tb.U))
    res = shooting.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    Phi = res["Phi"]
    assert np.allclose(Phi, Phi[0][None], atol=1e-13)
    J = shooting.jacobian(res)
    Rm = tor.rotation(tb.table, om[1:] / om[0])
    assert np.allclose(J, np.kron(Phi[0], Rm) - np.eye(J.shape[0]), atol=1e-12)


def _fd_jac(s, tr, om, Z0, tb, h=1e-6):
    n = Z0.size
    J = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = h
        rp = shooting.evaluate(s, tr, om, Z0 + e.reshape(Z0.shape), tables=tb)["R"].ravel()
        rm = shooting.evaluate(s, tr, om, Z0 - e.reshape(Z0.shape), tables=tb)["R"].ravel()
        J[:, j] = (rp - rm) / (2 * h)
    return J


def test_jacobian_matches_finite_differences_and_kron_form():
    s = tiny_system(n=2, seed=6, cubic=1.5, quad=0.4)
    om = np.array([1.0, GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 3)], S=[5], S1=24)
    tb = shooting.TorusTables(tr)
    Z0 = 0.3 * np.random.default_rng(1).normal(size=(4, tb.U))
    res = shooting.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    J = shooting.jacobian(res)
    assert np.allclose(J, shooting.jacobian_kron(res), atol=1e-13)
    assert np.allclose(J, _fd_jac(s, tr, om, Z0, tb), rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("d,e", [(2, 2), (2, 1), (3, 2)])
def test_residual_omega_derivative_matches_finite_differences(d, e):
    """Eq. (23)/(24): trajectory term for i <= e, rotation term for all i."""
    s = tiny_system(n=2, seed=8, cubic=1.0, quad=0.3, e=e)
    om = np.array([1.05, 1.05 * GOLDEN, 1.05 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=e, K=[np.arange(1, 3)] * (d - 1), S=[5] * (d - 1), S1=20)
    tb = shooting.TorusTables(tr)
    Z0 = 0.2 * np.random.default_rng(2).normal(size=(4, tb.U))
    res = shooting.evaluate(s, tr, om, Z0, omega_sens=True, tables=tb)
    dR = shooting.residual_domega(res, om, e)
    h = 1e-6
    for i in range(d):
        ei = np.zeros(d)
        ei[i] = h
        rp = shooting.evaluate(s, tr, om + ei, Z0, tables=tb)["R"].ravel()
        rm = shooting.evaluate(s, tr, om - ei, Z0, tables=tb)["R"].ravel()
        assert np.allclose(dR[:, i], (rp - rm) / (2 * h), rtol=1e-6, atol=1e-7), i


def test_newton_converges_quadratically_on_nonlinear_tiny():
    s = tiny_system(n=3, seed=9, cubic=0.5, quad=0.2)
    s.F *= 0.3
    om = np.array([0.45, 0.45 * GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 5)], S=[11], S1=48)
    tb = shooting.TorusTables(tr)
    Z, _, hist = shooting.solve(s, tr, om, np.zeros((6, tb.U)), tol_R=1e-13, tables=tb)
    assert hist[-1] < 1e-13
    # quadratic tail: r_{k+1} <= C r_k^2 with a bounded C over the last steps
    assert len(hist) <= 7
    assert hist[-2] < 10 * hist[-3] ** 2 and hist[-3] < 10 * hist[-4] ** 2


def test_d1_reduces_to_classical_shooting():
    """d = 1: R = Z(2 pi) - Z(0) (classical shooting); the discrete periodic orbit of a
    forced Duffing oscillator approaches the continuous one at second order."""
    from fse_inputs.systems import System
    k3 = 0.5
    s = System("duffing", np.eye(1), np.array([[0.1]]), np.eye(1),
               np.zeros((0, 3), np.int32), np.zeros(0),
               np.array([[0, 0, 0, 0]], np.int32), np.array([k3]), np.array([[0.4]]))
    om = np.array([0.7])

    def flow(z):
        def rhs(t, y):
            return [y[1], 0.4 * math.cos(om[0] * t) - 0.1 * y[1] - y[0] - k3 * y[0] ** 3]
        sol = solve_ivp(rhs, [0, 2 * math.pi / om[0]], [z[0], z[1] * om[0]],
                        rtol=1e-12, atol=1e-14)
        return np.array([sol.y[0, -1], sol.y[1, -1] / om[0]])

    defects = []
    for S1 in (128, 256):
        tr = Torus(d=1, e=1, K=[], S=[], S1=S1)
        tb = shooting.TorusTables(tr)
        assert tb.U == 1 and tb.Stilde == 1
        Z, _, hist = shooting.solve(s, tr, om, np.zeros((2, 1)), tol_R=1e-13, tables=tb)
        assert hist[-1] < 1e-13
        res = shooting.evaluate(s, tr, om, Z, tables=tb)
        assert np.allclose(res["R"], res["Z2pi"] - Z)
        defects.append(np.abs(flow(Z[:, 0]) - Z[:, 0]).max())
    assert 3.5 < defects[0] / defects[1] < 4.5


@pytest.mark.parametrize("d,e", [(2, 1), (3, 2)])
def test_bordered_newton_step_solves_its_linearisation(d, e):
    """d > e (Sec. 3.2): the step (dZ, d omega_u) satisfies the linearised residual
    R + J dZ + dR/d omega_u d omega_u = 0, with dR/d omega_u checked against central
    differences, and the phase condition of Eq. (18): [(I (x) nabla_i) Z0]^T dZ = 0."""
    s = tiny_system(n=2, seed=8, cubic=1.0, quad=0.3, e=e)
    om = np.array([1.05, 1.05 * GOLDEN, 1.05 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=e, K=[np.arange(1, 3)] * (d - 1), S=[5] * (d - 1), S1=20)
    tb = shooting.TorusTables(tr)
    Z0 = 0.2 * np.random.default_rng(2).normal(size=(4, tb.U))
    Z1, om1, r0 = shooting.newton_step(s, tr, om, Z0, tables=tb)
    res = shooting.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    J = shooting.jacobian(res)
    dRw = shooting.residual_domega(res, om, e, first=e + 1)
    h = 1e-6
    for u in range(d - e):
        ei = np.zeros(d)
        ei[e + u] = h
        rp = shooting.evaluate(s, tr, om + ei, Z0, tables=tb)["R"].ravel()
        rm = shooting.evaluate(s, tr, om - ei, Z0, tables=tb)["R"].ravel()
        assert np.allclose(dRw[:, u], (rp - rm) / (2 * h), rtol=1e-6, atol=1e-7)
    dZ, dw = (Z1 - Z0).ravel(), (om1 - om)[e:]
    assert np.allclose(om1[:e], om[:e])
    lin = res["R"].ravel() + J @ dZ + dRw @ dw
    assert np.linalg.norm(lin) < 1e-10 * max(1.0, np.linalg.norm(res["R"]))
    assert abs(r0 - np.linalg.norm(res["R"])) < 1e-14
    P = shooting.phase_rows(tb, Z0, e, d)
    assert np.abs(P @ dZ).max() < 1e-12 * np.linalg.norm(dZ) * np.abs(P).max()

"""Pins of the oracle's hyper-time FSE-Shooting (Sec. 3.4, Eq. FSES_T)."""
import numpy as np
import pytest

from _closed_forms import discrete_linear_torus
from fse_inputs import Torus, tiny_system
from oracle import hypertime as ht
from oracle import shooting

GOLDEN = (1 + 5 ** 0.5) / 2


def _case(d, nonlinear=True, seed=2, S=8):
    s = tiny_system(n=2, seed=seed, nonlinear=nonlinear, cubic=1.0, quad=0.3, e=d)
    om = np.array([0.8, 0.8 * GOLDEN, 0.8 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=d, K=[np.arange(1, 3)] * (d - 1), S=[S] * (d - 1), S1=32)
    return s, tr, shooting.TorusTables(tr), om


@pytest.mark.parametrize("d,S", [(2, 5), (2, 8), (3, 6)])
def test_residual_is_gamma_times_the_multifrequency_residual(d, S):
    """zbar(0) = Gamma Z(0): R_ht = Gamma R_mf (Gamma^-1 Gamma = I), with S~ = U~ and S~ > U~."""
    s, tr, tb, om = _case(d, S=S)
    Z0 = 0.2 * np.random.default_rng(3).normal(size=(4, tb.U))
    mf = shooting.evaluate(s, tr, om, Z0, tables=tb)
    h = ht.evaluate(s, tr, om, Z0 @ tb.G.T, tables=tb)
    assert np.allclose(h["R"], mf["R"] @ tb.G.T, rtol=1e-12, atol=1e-13)
    # A is a projection onto the band-limited samples, rotated: A^k = Gamma R^k Gamma^-1
    A = h["A"]
    assert np.allclose(A @ A, tb.G @ (mf["Rrot"] @ mf["Rrot"]) @ tb.Gi, atol=1e-12)


def test_jacobian_matches_finite_differences():
    s, tr, tb, om = _case(2, S=5)
    z0 = 0.2 * np.random.default_rng(4).normal(size=(4, tb.Stilde))
    res = ht.evaluate(s, tr, om, z0, sens=True, tables=tb)
    J = ht.jacobian(res)
    h = 1e-6
    fd = np.empty_like(J)
    for c in range(J.shape[1]):
        e = np.zeros(J.shape[1])
        e[c] = h
        rp = ht.evaluate(s, tr, om, z0 + e.reshape(z0.shape), tables=tb)["R"].ravel()
        rm = ht.evaluate(s, tr, om, z0 - e.reshape(z0.shape), tables=tb)["R"].ravel()
        fd[:, c] = (rp - rm) / (2 * h)
    assert np.allclose(J, fd, rtol=1e-6, atol=1e-7)


def test_linear_closed_form_torus_sampled_is_the_solution():
    s, tr, tb, om = _case(2, nonlinear=False, S=8)
    Zs = discrete_linear_torus(s, om, tr.S1, tb.table, tb.U)
    zs = Zs @ tb.G.T
    res = ht.evaluate(s, tr, om, zs, tables=tb)
    assert np.linalg.norm(res["R"]) < 1e-12 * np.linalg.norm(zs)
    z1, r0 = ht.newton_step(s, tr, om, np.zeros_like(zs), tables=tb)
    assert r0 > 1e-3
    assert np.abs(z1 - zs).max() < 1e-12 * np.abs(zs).max()


def test_nonlinear_solution_is_the_sampled_multifrequency_torus():
    s, tr, tb, om = _case(2, S=8)
    s.F *= 0.5
    Zm, _, hm = shooting.solve(s, tr, om, np.zeros((4, tb.U)), tol_R=1e-13, tables=tb)
    zh, hh = ht.solve(s, tr, om, np.zeros((4, tb.Stilde)), tol_R=1e-13, tables=tb)
    assert hm[-1] < 1e-13 and hh[-1] < 1e-13
    assert np.abs(zh - Zm @ tb.G.T).max() < 1e-10 * np.abs(zh).max()


def test_unknown_frequency_border_matches_the_multi_frequency_step():
    """d > e with S~ = U~ (Gamma invertible): the bordered hyper-time step from zbar = Gamma Z is
    Gamma times the multi-frequency bordered step, with the same omega_u update; the border
    column matches central differences in omega_2."""
    from oracle import hypertime as oht
    s = tiny_system(n=2, seed=8, cubic=1.0, quad=0.3, e=1)
    tr = Torus(d=2, e=1, K=[np.arange(1, 3)], S=[5], S1=20)
    tb = shooting.TorusTables(tr)
    assert tb.Stilde == tb.U
    om = np.array([1.05, 1.05 * (1 + 5 ** 0.5) / 2])
    Z0 = 0.2 * np.random.default_rng(2).normal(size=(4, tb.U))
    Z1, om1, r1 = shooting.newton_step(s, tr, om, Z0, tables=tb)
    zb1, omh, rh = oht.newton_step(s, tr, om, Z0 @ tb.G.T, tables=tb)
    assert np.allclose(zb1, Z1 @ tb.G.T, rtol=1e-9, atol=1e-11)
    assert np.allclose(omh, om1, rtol=1e-11)
    res = oht.evaluate(s, tr, om, Z0 @ tb.G.T, tables=tb)
    B, P = oht.border(res, om, 1, Z0 @ tb.G.T)
    h = 1e-6
    e2 = np.array([0.0, h])
    fd = (oht.evaluate(s, tr, om + e2, Z0 @ tb.G.T, tables=tb)["R"]
          - oht.evaluate(s, tr, om - e2, Z0 @ tb.G.T, tables=tb)["R"]).ravel() / (2 * h)
    assert np.allclose(B[:, 0], fd, rtol=1e-7, atol=1e-9)


def test_bordered_solve_returns_the_unknown_frequency_and_reaches_the_van_der_pol_torus():
    """d > e: solve() carries omega_u through every bordered step.  On the forced van der Pol
    oscillator (omega_2 the free limit-cycle frequency) the hyper-time solution, started from
    the sampled averaging iterate, has the free frequency of the multi-frequency solution and
    its samples are that torus up to the phase along omega_2 (compared through amplitudes)."""
    import math
    from _velocity_systems import van_der_pol
    from fse_inputs.systems import place_harmonics
    s = van_der_pol(mu=0.2)
    w1 = 2.3
    tr = Torus(d=2, e=1, K=[np.arange(1, 6)], S=[11], S1=96)
    tb = shooting.TorusTables(tr)
    A = 0.5 / (1 - w1 ** 2)
    Z0 = place_harmonics(tb.table, [((0,), np.array([A, 0.0], complex)), ((1,), np.array([2.0, 2j / w1]))],
                         1, tb.U)
    om = np.array([w1, 1.0])
    Zm, omm, hm = shooting.solve(s, tr, om, Z0, tol_R=1e-11, max_newton=25, tables=tb)
    out = ht.solve(s, tr, om, Z0 @ tb.G.T, tol_R=1e-11, max_newton=25, tables=tb)
    assert len(out) == 3
    zh, omh, hist = out
    assert hm[-1] < 1e-11 and hist[-1] < 1e-11
    assert omh[0] == om[0]
    assert abs(omh[1] - omm[1]) < 1e-9
    Zh = zh @ tb.Gi.T
    amp = lambda Z, l: math.hypot(Z[0, 2 * l + 1], Z[0, 2 * l + 2])
    for l in range(tb.U // 2):
        assert abs(amp(Zh, l) - amp(Zm, l)) < 1e-8

"""Pins of the oracle's multiple FSE-Shooting (the paper's first recommendation, classical
multiple-shooting reading)."""
import numpy as np
import pytest

from fse_inputs import Torus, tiny_system
from _closed_forms import discrete_linear_sections as _linear_sections
from oracle import multiple as mult
from oracle import shooting

GOLDEN = (1 + 5 ** 0.5) / 2


def _case(nonlinear=True, seed=2, S=8, S1=48):
    s = tiny_system(n=2, seed=seed, nonlinear=nonlinear, cubic=1.0, quad=0.3, e=2)
    om = np.array([0.8, 0.8 * GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 3)], S=[S], S1=S1)
    return s, tr, shooting.TorusTables(tr), om


def test_one_segment_is_fse_shooting():
    s, tr, tb, om = _case()
    Z = 0.2 * np.random.default_rng(3).normal(size=(4, tb.U))
    single = shooting.evaluate(s, tr, om, Z, sens=True, tables=tb)
    one = mult.evaluate(s, tr, om, Z[None], 1, sens=True, tables=tb)
    assert np.allclose(one["R"][0], single["R"], rtol=1e-13, atol=1e-14)
    assert np.allclose(mult.jacobian(one), shooting.jacobian(single), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("M", [2, 3, 4])
def test_linear_sections_are_the_closed_form(M):
    s, tr, tb, om = _case(nonlinear=False)
    Zc = _linear_sections(s, om, tr.S1, tb.table, tb.U, M)
    res = mult.evaluate(s, tr, om, Zc, M, tables=tb)
    assert np.abs(res["R"]).max() < 1e-12 * np.abs(Zc).max()
    Z1, r0 = mult.newton_step(s, tr, om, np.zeros_like(Zc), M, tables=tb)
    assert r0 > 1e-3
    assert np.abs(Z1 - Zc).max() < 1e-12 * np.abs(Zc).max()


def test_jacobian_matches_finite_differences():
    s, tr, tb, om = _case(S=5, S1=24)
    M = 3
    Zs = 0.2 * np.random.default_rng(4).normal(size=(M, 4, tb.U))
    J = mult.jacobian(mult.evaluate(s, tr, om, Zs, M, sens=True, tables=tb))
    h = 1e-6
    fd = np.empty_like(J)
    for c in range(J.shape[1]):
        e = np.zeros(J.shape[1])
        e[c] = h
        rp = mult.evaluate(s, tr, om, Zs + e.reshape(Zs.shape), M, tables=tb)["R"].ravel()
        rm = mult.evaluate(s, tr, om, Zs - e.reshape(Zs.shape), M, tables=tb)["R"].ravel()
        fd[:, c] = (rp - rm) / (2 * h)
    assert np.allclose(J, fd, rtol=1e-6, atol=1e-7)


def test_nonlinear_section_zero_is_the_single_shooting_torus():
    """Both forms solve the same torus; they differ by how the truncated Fourier basis
    represents the intermediate sections, so section 0 agrees to the truncation level."""
    s, tr, tb, om = _case(S=8)
    s.F *= 0.5
    Z1, _, h1 = shooting.solve(s, tr, om, np.zeros((4, tb.U)), tol_R=1e-12, tables=tb)
    M = 2
    Zm, hm = mult.solve(s, tr, om, np.zeros((M, 4, tb.U)), M, tol_R=1e-12, tables=tb)
    assert h1[-1] < 1e-12 and hm[-1] < 1e-12
    err = np.abs(Zm[0] - Z1).max() / np.abs(Z1).max()
    print("section 0 vs single shooting", err)
    assert err < 1e-3


def test_unknown_frequency_bordered_step():
    """d > e: M = 1 reproduces the single-shooting bordered Newton step, dR/d omega_u of the
    segments matches central differences, and the forced van der Pol torus solved with two
    segments has the single-shooting free frequency and section 0."""
    from _velocity_systems import van_der_pol
    from fse_inputs.systems import place_harmonics
    s = tiny_system(n=2, seed=8, cubic=1.0, quad=0.3, e=1)
    tr = Torus(d=2, e=1, K=[np.arange(1, 3)], S=[5], S1=20)
    tb = shooting.TorusTables(tr)
    om = np.array([1.05, 1.05 * (1 + 5 ** 0.5) / 2])
    Z0 = 0.2 * np.random.default_rng(2).normal(size=(4, tb.U))
    Zm, omm, rm = mult.newton_step(s, tr, om, Z0[None], 1, tables=tb)
    Zs, oms, rs = shooting.newton_step(s, tr, om, Z0, tables=tb)
    assert abs(rm - rs) < 1e-13 * rs
    assert np.allclose(Zm[0], Zs, rtol=1e-10, atol=1e-12) and np.allclose(omm, oms, rtol=1e-12)
    M = 2
    Zz = 0.2 * np.random.default_rng(3).normal(size=(M, 4, tb.U))
    res = mult.evaluate(s, tr, om, Zz, M, tables=tb)
    B = mult.residual_domega_u(res, om, 1, Zz)
    h = 1e-6
    e2 = np.array([0.0, h])
    fd = (mult.evaluate(s, tr, om + e2, Zz, M, tables=tb)["R"]
          - mult.evaluate(s, tr, om - e2, Zz, M, tables=tb)["R"]).ravel() / (2 * h)
    assert np.allclose(B[:, 0], fd, rtol=1e-7, atol=1e-9)
    v = van_der_pol(mu=0.2)
    w1 = 2.3
    trv = Torus(d=2, e=1, K=[np.arange(1, 8)], S=[16], S1=128)
    tbv = shooting.TorusTables(trv)
    A = 0.5 / (1 - w1 ** 2)
    Zi = place_harmonics(tbv.table, [((0,), np.array([A, 0.0], complex)), ((1,), np.array([2.0, 2j / w1]))],
                         1, tbv.U)
    Z1, om1, _ = shooting.solve(v, trv, np.array([w1, 1.0]), Zi, tol_R=1e-11, max_newton=25, tables=tbv)
    # second section from half a period of the single-shooting torus
    zb = Z1 @ tbv.G.T
    from oracle import newmark
    half = np.stack([newmark.integrate(v, om1, 128, tbv.phases[:, j], zb[:, j], steps=64)["zT"]
                     for j in range(tbv.Stilde)], axis=1)
    import oracle.torus as tor
    Zh = (half @ tbv.Gi.T) @ tor.rotation(tbv.table, om1[1:] / om1[0] / 2).T
    Zm2, omm2, hist = mult.solve(v, trv, np.array([w1, 0.999]), np.stack([Z1, Zh]), 2, tol_R=1e-10,
                                     max_newton=10, tables=tbv)
    assert hist[-1] < 1e-10
    assert abs(omm2[1] - om1[1]) < 1e-9
    # the phase of the free oscillation is fixed only relative to each Newton path: compare the
    # amplitude of every harmonic pair, which a shift of phi_2 leaves unchanged, to the truncation
    amp = lambda Z: np.hypot(Z[:, 1::2], Z[:, 2::2])
    assert np.allclose(amp(Zm2[0]), amp(Z1), atol=1e-4)

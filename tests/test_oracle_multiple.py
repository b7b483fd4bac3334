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

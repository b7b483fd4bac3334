"""Pins of the oracle's pseudo-arclength continuation in omega_1 (App. C, Sec. 3.2.1)."""
import numpy as np
import pytest

from _closed_forms import discrete_linear_torus
from fse_inputs import Torus, tiny_system
from fse_inputs.systems import System
from oracle import continuation as cont
from oracle import shooting

GOLDEN = (1 + 5 ** 0.5) / 2


def duffing(k3=0.5, F=0.15, D=0.1):
    """q'' + D q' + q + k3 q^3 = F cos(t): hardening, with two folds at these values."""
    return System("duffing", np.eye(1), np.array([[D]]), np.eye(1), np.zeros((0, 3), np.int32),
                  np.zeros(0), np.array([[0, 0, 0, 0]], np.int32), np.array([k3]), np.array([[F]]))


@pytest.mark.parametrize("d,e", [(1, 1), (2, 2), (2, 1), (3, 2), (3, 3)])
def test_dR_dp_matches_finite_differences_along_frequency_conditions(d, e):
    """dR/dp (p = omega_1; omega_j = rho_j p for j <= e, omega_u held) against
    central differences of R along that same direction."""
    s = tiny_system(n=2, seed=8, cubic=1.0, quad=0.3, e=e)
    if d == 3 and e == 3:
        s.F[2, 0] = 0.5
    om = np.array([1.05, 1.05 * GOLDEN, 1.05 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=e, K=[np.arange(1, 3)] * (d - 1), S=[5] * (d - 1), S1=20)
    tb = shooting.TorusTables(tr)
    Z0 = 0.2 * np.random.default_rng(2).normal(size=(4, tb.U))
    res = shooting.evaluate(s, tr, om, Z0, omega_sens=True, tables=tb)
    dRp = cont.residual_dp(res, om, e)
    h = 1e-6
    rp = shooting.evaluate(s, tr, cont.frequencies(om, om[0] + h, e), Z0, tables=tb)["R"].ravel()
    rm = shooting.evaluate(s, tr, cont.frequencies(om, om[0] - h, e), Z0, tables=tb)["R"].ravel()
    fd = (rp - rm) / (2 * h)
    assert np.allclose(dRp, fd, rtol=1e-6, atol=1e-7)
    # the frequency conditions keep the forcing ratios and leave omega_u alone
    om2 = cont.frequencies(om, 1.3, e)
    assert np.allclose(om2[:e] / om2[0], om[:e] / om[0]) and np.all(om2[e:] == om[e:])


def test_linear_path_is_the_closed_form_torus_at_every_point():
    """Linear system, d = e = 2: each point of the arclength path is the discrete
    closed-form torus at its own omega_1, reached by one corrector iteration, and
    omega_1 increases monotonically (no folds without nonlinearity)."""
    s = tiny_system(n=3, seed=2, nonlinear=False, e=2)
    om0 = np.array([1.3, 1.3 * GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 4)], S=[8], S1=64)
    tb = shooting.TorusTables(tr)
    Z0 = discrete_linear_torus(s, om0, tr.S1, tb.table, tb.U)
    path = cont.arclength(s, tr, om0, Z0, 0.05, 6, tables=tb, tol_R=1e-11)
    ps = [p["omega"][0] for p in path]
    assert np.all(np.diff(ps) > 0)
    for p in path[1:]:
        Zc = discrete_linear_torus(s, p["omega"], tr.S1, tb.table, tb.U)
        assert np.abs(p["Z"] - Zc).max() < 1e-10 * np.abs(Zc).max()
        assert np.isclose(p["omega"][1] / p["omega"][0], GOLDEN)
        # a linear residual in Z: the corrector's first step lands within the O(s^2)
        # curvature in p and the second one on the branch
        assert len(p["hist"]) <= 4


def test_duffing_path_turns_at_both_folds():
    """Forced hardening Duffing oscillator (d = 1, classical shooting): the path runs up
    the resonant branch, turns at the upper fold, comes back along the middle branch,
    turns at the lower fold and continues on the upper-frequency branch.  At each turn
    dp changes sign and det(dR/dZ) changes sign with it; every point solves R = 0; the
    corrector lands on the hyperplane t_j^T (x - x_j) = s_j of Eq. (C3)."""
    s = duffing()
    tr = Torus(d=1, e=1, K=[], S=[], S1=64)
    tb = shooting.TorusTables(tr)
    om0 = np.array([0.6])
    Z0, _, h = shooting.solve(s, tr, om0, np.zeros((2, 1)), tol_R=1e-12, tables=tb)
    path = cont.arclength(s, tr, om0, Z0, 0.15, 26, tables=tb, tol_R=1e-10)
    tp = np.array([p["t"][-1] for p in path])
    dets = []
    for p in path:
        res = shooting.evaluate(s, tr, p["omega"], p["Z"], sens=True, tables=tb)
        assert np.linalg.norm(res["R"]) < 1e-10
        dets.append(np.linalg.det(shooting.jacobian(res)))
    dets = np.array(dets)
    turns = np.flatnonzero(np.sign(tp[1:]) != np.sign(tp[:-1]))
    assert len(turns) == 2, tp
    assert np.array_equal(np.flatnonzero(np.sign(dets[1:]) != np.sign(dets[:-1])), turns)
    # the upper fold lies above the linear resonance (hardening), the lower one below it
    w_up, w_lo = path[turns[0]]["omega"][0], path[turns[1]]["omega"][0]
    assert 1.0 < w_lo < w_up
    for a, b in zip(path[:-1], path[1:]):
        xa = np.concatenate([a["Z"].ravel(), [a["omega"][0]]])
        xb = np.concatenate([b["Z"].ravel(), [b["omega"][0]]])
        assert abs(a["t"] @ (xb - xa) - b["s"]) < 1e-12
        assert abs(a["t"] @ (xb - b["x_pred"])) < 1e-12
        assert abs(np.linalg.norm(b["t"]) - 1.0) < 1e-14

"""Pins of the oracle's Lyapunov exponents (App. F)."""
import math

import numpy as np

from fse_inputs import Torus, tiny_system
from oracle import lyapunov, shooting
from oracle import torus as tor

GOLDEN = (1 + 5 ** 0.5) / 2


def _converged(s, tr, om):
    tb = shooting.TorusTables(tr)
    Z, _, hist = shooting.solve(s, tr, om, np.zeros((2 * s.n, tb.U)), tol_R=1e-12, tables=tb)
    assert hist[-1] < 1e-12
    res = shooting.evaluate(s, tr, om, Z, sens=True, tables=tb)
    return res, tb


def test_sum_of_exponents_equals_mean_log_det():
    """Exact for any system: prod |R_hh| = |det Psi_i| at every step of the QR sweep."""
    s = tiny_system(n=3, seed=9, cubic=0.5, quad=0.2)
    s.F *= 0.3
    om = np.array([0.45, 0.45 * GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 5)], S=[11], S1=48)
    res, tb = _converged(s, tr, om)
    N = 200
    sig, _, _ = lyapunov.exponents(res["Phi"], om, tb, N_Ly=N)
    T1 = 2 * math.pi / om[0]
    rho = om[1:] / om[0]
    logdet = 0.0
    for i in range(1, N + 1):
        Psi = lyapunov.interpolated_transition(res["Phi"], om, tb, 2 * math.pi * (i - 1) * rho)
        logdet += math.log(abs(np.linalg.det(Psi)))
    assert abs(sig.sum() - logdet / (N * T1)) < 1e-10 * max(1.0, abs(sig.sum()))
    # the nonlinear transition matrix really varies over the torus
    assert np.abs(res["Phi"] - res["Phi"][0][None]).max() > 1e-4


def test_linear_exponents_are_log_moduli_of_trapezoidal_map():
    """Linear system: Psi is constant; exponents -> log|mu|/T1 with
    mu = ((1 + h l/2)/(1 - h l/2))^S1 for the eigenvalues l of the first-order
    system in phi_1-time (average acceleration = trapezoidal rule)."""
    s = tiny_system(n=2, seed=4, nonlinear=False, zeta=0.05)
    om = np.array([0.9, 0.9 * GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 3)], S=[5], S1=32)
    tb = shooting.TorusTables(tr)
    res = shooting.evaluate(s, tr, om, np.zeros((4, tb.U)), sens=True, tables=tb)
    w1 = om[0]
    n = 2
    Minv = np.linalg.inv(s.M)
    A = np.block([[np.zeros((n, n)), np.eye(n)], [-Minv @ s.K / w1 ** 2, -Minv @ s.D / w1]])
    lam = np.linalg.eigvals(A)
    h = 2 * math.pi / tr.S1
    mu = ((1 + h * lam / 2) / (1 - h * lam / 2)) ** tr.S1
    Psi = lyapunov.transition_samples(res["Phi"], w1)[0]
    assert np.allclose(np.sort_complex(np.linalg.eigvals(Psi)), np.sort_complex(mu), atol=1e-11)
    T1 = 2 * math.pi / w1
    # generic start basis: from Q0 = I the start plane of this nearly decoupled
    # system is ~87 degrees off the dominant subspace and needs ~200 sweeps
    Q0, _ = np.linalg.qr(np.random.default_rng(11).normal(size=(4, 4)))
    _, sig, _ = lyapunov.exponents(res["Phi"], om, tb, N_Ly=3000, Q0=Q0)
    expect = np.sort(np.log(np.abs(mu)) / T1)[::-1]
    # complex pairs share a modulus: compare pair sums tightly, entries loosely
    assert abs(sig.sum() - expect.sum()) < 1e-11
    assert np.allclose(sig, expect, atol=2e-3 * abs(expect).max())


def test_continuous_limit_sum_is_minus_trace():
    """Resolved modes: sum sigma -> -tr(M^-1 D) (phase-space divergence), O(h^2)."""
    s = tiny_system(n=2, seed=4, nonlinear=False, zeta=0.05)
    om = np.array([0.9, 0.9 * GOLDEN])
    target = -np.trace(np.linalg.solve(s.M, s.D))
    errs = []
    for S1 in (128, 256):
        tr = Torus(d=2, e=2, K=[np.arange(1, 3)], S=[5], S1=S1)
        tb = shooting.TorusTables(tr)
        res = shooting.evaluate(s, tr, om, np.zeros((4, tb.U)), sens=True, tables=tb)
        sig, _, _ = lyapunov.exponents(res["Phi"], om, tb, N_Ly=50)
        errs.append(abs(sig.sum() - target))
    assert errs[1] < 1e-3 * abs(target)
    assert errs[0] / errs[1] > 3.5


def test_interpolation_reproduces_samples():
    """Psi(phi~_s) interpolated at the grid equals the sampled Psi_s (band-limited basis)."""
    s = tiny_system(n=2, seed=6, cubic=1.0, quad=0.3)
    om = np.array([0.5, 0.5 * GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 3)], S=[5], S1=24)
    tb = shooting.TorusTables(tr)
    Z0 = 0.2 * np.random.default_rng(3).normal(size=(4, tb.U))
    res = shooting.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    Psi = lyapunov.transition_samples(res["Phi"], om[0])
    ang = tor.sample_angles(tr.S)
    for s_ in range(5):
        P = lyapunov.interpolated_transition(res["Phi"], om, tb, ang[:, s_])
        assert np.allclose(P, Psi[s_], atol=1e-12)

"""Pins of the oracle's matrix-free Newton-Krylov step (Eq. 22 applied to vectors, GMRES)."""
import numpy as np
import pytest

from _closed_forms import discrete_linear_torus
from fse_inputs import Torus, tiny_system
from oracle import krylov
from oracle import shooting

GOLDEN = (1 + 5 ** 0.5) / 2


def _case(d, nonlinear=True, seed=2, S1=48):
    s = tiny_system(n=3, seed=seed, nonlinear=nonlinear, cubic=1.0, quad=0.3, e=d)
    om = np.array([0.8, 0.8 * GOLDEN, 0.8 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=d, K=[np.arange(1, 4)] * (d - 1), S=[8] * (d - 1), S1=S1)
    tb = shooting.TorusTables(tr)
    return s, tr, tb, om


@pytest.mark.parametrize("d", [2, 3])
def test_jacobian_apply_is_the_dense_jacobian(d):
    s, tr, tb, om = _case(d)
    rng = np.random.default_rng(4)
    Z0 = 0.2 * rng.normal(size=(6, tb.U))
    res = shooting.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    J = shooting.jacobian(res)
    for _ in range(3):
        v = rng.normal(size=(6, tb.U))
        assert np.allclose(krylov.jacobian_apply(res, v).ravel(), J @ v.ravel(), rtol=1e-12, atol=1e-12)


def test_harmonic_preconditioner_is_exact_for_a_linear_system():
    """Linear system: every Phi_s is the same matrix, so P = J; P^-1 J v = v, and
    preconditioned GMRES solves the Newton system in one iteration."""
    s, tr, tb, om = _case(2, nonlinear=False)
    Zs = discrete_linear_torus(s, om, tr.S1, tb.table, tb.U)
    Z0 = np.zeros_like(Zs)
    res = shooting.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    blocks = krylov.harmonic_blocks(res)
    v = np.random.default_rng(5).normal(size=Z0.shape)
    assert np.allclose(krylov.precondition(blocks, krylov.jacobian_apply(res, v)), v, rtol=1e-11, atol=1e-11)
    Z1, r0, its, rel = krylov.newton_krylov_step(s, tr, om, Z0, rtol=1e-12, tables=tb)
    assert its == 1 and rel < 1e-12
    assert np.abs(Z1 - Zs).max() < 1e-11 * np.abs(Zs).max()
    # the unpreconditioned iteration needs many more steps for the same system
    _, _, its_u, rel_u = krylov.newton_krylov_step(s, tr, om, Z0, rtol=1e-12, precond=False, tables=tb)
    assert rel_u < 1e-12 and its_u > 5


@pytest.mark.parametrize("precond", [True, False])
def test_gmres_correction_meets_its_tolerance(precond):
    """Nonlinear system: the GMRES correction satisfies ||R + J dZ|| <= rtol ||R|| with the
    dense J, and agrees with the dense solve to the tolerance's accuracy."""
    s, tr, tb, om = _case(2)
    Z0 = 0.2 * np.random.default_rng(6).normal(size=(6, tb.U))
    res = shooting.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    J = shooting.jacobian(res)
    R = res["R"].ravel()
    for rtol in (1e-4, 1e-10):
        Z1, r0, its, rel = krylov.newton_krylov_step(s, tr, om, Z0, rtol=rtol, restart=10, precond=precond,
                                                     tables=tb)
        dZ = (Z1 - Z0).ravel()
        assert np.linalg.norm(R + J @ dZ) <= 1.0001 * rtol * np.linalg.norm(R)
        dref = np.linalg.solve(J, -R)
        assert np.linalg.norm(dZ - dref) <= 1e3 * rtol * np.linalg.norm(dref)


def test_newton_krylov_reaches_the_dense_newton_torus():
    s = tiny_system(n=3, seed=9, cubic=0.5, quad=0.2)
    s.F *= 0.3
    om = np.array([0.45, 0.45 * GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 5)], S=[11], S1=48)
    tb = shooting.TorusTables(tr)
    Zd, _, hist = shooting.solve(s, tr, om, np.zeros((6, tb.U)), tol_R=1e-13, tables=tb)
    Z = np.zeros((6, tb.U))
    its = []
    for _ in range(8):
        Z, r0, it, rel = krylov.newton_krylov_step(s, tr, om, Z, rtol=1e-12, tables=tb)
        its.append(it)
        if r0 < 1e-13:
            break
    res = shooting.evaluate(s, tr, om, Z, tables=tb)
    assert np.linalg.norm(res["R"]) < 1e-12
    assert np.abs(Z - Zd).max() < 1e-10 * np.abs(Zd).max()

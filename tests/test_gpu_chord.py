"""GPU simplified (chord) Newton-Krylov steps against the oracle.

A chord step takes the residual at the new point from the states alone and solves with the
Jacobian stored by the last matrix-free evaluation, possibly at another Z(0) and omega.  Bar:
the reported ||R|| within 1e-10 of the oracle's residual at the new point; the correction meets
||R_new + J_stored dZ|| <= rtol ||R_new|| with the oracle's dense Jacobian of the stored point;
a run of chord steps after a frequency step ends on a root of the oracle's residual and on
the oracle's Newton torus; J v keeps the stored rotation after evaluations elsewhere.
"""
import numpy as np
import pytest

from fse_inputs import Torus, tiny_system
from fse_inputs.systems import banded_lumped_system
from oracle import shooting as osh

pytestmark = pytest.mark.gpu
GOLDEN = (1 + 5 ** 0.5) / 2
RTOL = 1e-10


def fse():
    import paper_2508_06302_amd as m
    return m


def rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def log(msg):
    print(msg, flush=True)


def _tiny(d=2):
    s = tiny_system(n=3, seed=2, cubic=1.0, quad=0.3, e=d)
    om = np.array([0.8, 0.8 * GOLDEN, 0.8 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=d, K=[np.arange(1, 4)] * (d - 1), S=[8] * (d - 1), S1=48)
    return s, tr, osh.TorusTables(tr), om


def _banded():
    s = banded_lumped_system(n=37, bw=20, seed=3)
    tr = Torus(d=2, e=2, K=[np.arange(1, 4)], S=[8], S1=48)
    return s, tr, osh.TorusTables(tr), np.array([1.1, 1.1 * GOLDEN])


@pytest.mark.parametrize("case", ["tiny", "wide"])
@pytest.mark.parametrize("precond", [True, False])
def test_chord_step_solves_with_the_stored_jacobian(case, precond, monkeypatch):
    """Stored J at (omega_a, Z_a); chord step at (omega_b, Z_b): R is that of the new point,
    the correction solves J(omega_a, Z_a) dZ = -R(omega_b, Z_b)."""
    import torch
    if case == "wide":
        monkeypatch.setenv("FSE_KERNELS", "wide")
        s, tr, tb, om_a = _banded()
        scale = 0.3
    else:
        s, tr, tb, om_a = _tiny()
        scale = 0.2
    rng = np.random.default_rng(11)
    Z_a = scale * rng.normal(size=(2 * s.n, tb.U))
    Z_b = Z_a + 0.02 * scale * rng.normal(size=Z_a.shape)
    om_b = om_a * 1.004
    J_a = osh.jacobian(osh.evaluate(s, tr, om_a, Z_a, sens=True, tables=tb))
    R_b = osh.evaluate(s, tr, om_b, Z_b, tables=tb)["R"].ravel()
    ctx = fse().fse_init_torus(s, tr)
    fse().fse_shooting_residual_matfree(ctx, om_a, Z_a)
    for rtol in (1e-4, 1e-10):
        Zg = torch.tensor(Z_b, dtype=torch.float64, device="cuda")
        rn, its, relres = fse().fse_newton_krylov_chord_step(ctx, om_b, Zg, rtol=rtol, restart=12, maxit=400,
                                                             precond=precond)
        dZ = Zg.cpu().numpy().ravel() - Z_b.ravel()
        lin = np.linalg.norm(R_b + J_a @ dZ) / np.linalg.norm(R_b)
        log(f"chord {case} precond={precond} rtol={rtol:g}: {its} GMRES iterations, reported {relres:.2e}, "
            f"with the oracle's stored J {lin:.2e}")
        assert abs(rn - np.linalg.norm(R_b)) < RTOL * np.linalg.norm(R_b)
        assert relres <= rtol
        assert lin <= 1.001 * rtol + 1e-13


def test_jacobian_apply_keeps_the_stored_rotation():
    """A residual evaluated elsewhere (other omega, so other rotation angles) leaves J v as it
    was: the stored J keeps the rotation of its own evaluation."""
    import torch
    s, tr, tb, om = _tiny()
    rng = np.random.default_rng(3)
    Z0 = 0.2 * rng.normal(size=(6, tb.U))
    v = torch.tensor(rng.normal(size=(6, tb.U)), dtype=torch.float64, device="cuda")
    ctx = fse().fse_init_torus(s, tr)
    fse().fse_shooting_residual_matfree(ctx, om, Z0)
    Jv0 = fse().fse_jacobian_apply(ctx, v).cpu().numpy()
    fse().fse_shooting_residual_jacobian(ctx, om[None] * 1.3, Z0[None], want_J=False)
    Jv1 = fse().fse_jacobian_apply(ctx, v).cpu().numpy()
    assert np.array_equal(Jv0, Jv1)
    ref = osh.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    assert rel(Jv1.ravel(), osh.jacobian(ref) @ v.cpu().numpy().ravel()) < RTOL


def test_chord_iteration_after_a_frequency_step_reaches_the_oracle_torus():
    """Solve at omega_a by Newton-Krylov, step omega by 1 %, then chord steps only (the J of the
    old point): linear convergence to a root of the oracle's residual, the oracle's torus."""
    import torch
    s, tr, tb, om_a = _tiny()
    Zi = np.zeros((6, tb.U))
    Za, _, _ = osh.solve(s, tr, om_a, Zi, tol_R=1e-12, tables=tb)
    om_b = om_a * 1.01
    Zb, _, _ = osh.solve(s, tr, om_b, Za, tol_R=1e-12, tables=tb)
    ctx = fse().fse_init_torus(s, tr)
    Zg = torch.tensor(Za, dtype=torch.float64, device="cuda")
    fse().fse_newton_krylov_step(ctx, om_a, Zg, rtol=1e-12, restart=40, maxit=400)
    hist = []
    for _ in range(40):
        rn, its, _ = fse().fse_newton_krylov_chord_step(ctx, om_b, Zg, rtol=1e-12, restart=40, maxit=400)
        hist.append(rn)
        if rn < 1e-11:
            break
    log(f"chord residuals after a 1 % frequency step: {['%.1e' % h for h in hist]}")
    assert hist[-1] < 1e-11
    rates = [hist[i + 1] / hist[i] for i in range(len(hist) - 1) if hist[i] > 1e-9]
    assert rates and max(rates) < 0.5
    Zgpu = Zg.cpu().numpy()
    assert np.linalg.norm(osh.evaluate(s, tr, om_b, Zgpu, tables=tb)["R"]) < 1e-10
    assert rel(Zgpu, Zb) < 1e-9


def test_chord_error_paths():
    import torch
    s, tr, tb, om = _tiny()
    ctx = fse().fse_init_torus(s, tr)
    Zg = torch.zeros((6, tb.U), dtype=torch.float64, device="cuda")
    with pytest.raises(fse().FseError, match="FSE_E_INVAL"):
        fse().fse_newton_krylov_chord_step(ctx, om, Zg)
    fse().fse_shooting_residual_matfree(ctx, om, Zg)
    fse().fse_newton_krylov_chord_step(ctx, om, Zg)
    # a call that writes the sensitivity buffer discards the stored Jacobian
    fse().fse_lyapunov(ctx, om, Zg, 4)
    with pytest.raises(fse().FseError, match="FSE_E_INVAL"):
        fse().fse_newton_krylov_chord_step(ctx, om, Zg)
    with pytest.raises(ValueError):
        fse().fse_newton_krylov_chord_step(ctx, om, Zg.float())
    s3 = tiny_system(n=3, seed=8, cubic=1.0, quad=0.3, e=1)
    tr3 = Torus(d=2, e=1, K=[np.arange(1, 4)], S=[8], S1=48)
    ctx3 = fse().fse_init_torus(s3, tr3)
    Z3 = torch.zeros((6, osh.TorusTables(tr3).U), dtype=torch.float64, device="cuda")
    with pytest.raises(fse().FseError, match="FSE_E_UNSUPPORTED"):
        fse().fse_newton_krylov_chord_step(ctx3, np.array([1.05, 1.05 * GOLDEN]), Z3)

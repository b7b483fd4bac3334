"""GPU hyper-time FSE-Shooting (Sec. 3.4, Eq. FSES_T) against the oracle.

Bar: residual and Jacobian within 1e-10 normwise relative of the oracle; the hyper-time
residual at Gamma Z(0) is Gamma times the GPU's multi-frequency residual; converged
hyper-time tori (||R|| < 1e-12) equal the oracle's and the sampled multi-frequency torus.
"""
import numpy as np
import pytest

from fse_inputs import Torus, tiny_system, workload
from oracle import hypertime as oht
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


def _case(d, S, seed=2):
    s = tiny_system(n=2, seed=seed, cubic=1.0, quad=0.3, e=d)
    om = np.array([0.8, 0.8 * GOLDEN, 0.8 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=d, K=[np.arange(1, 3)] * (d - 1), S=[S] * (d - 1), S1=32)
    return s, tr, osh.TorusTables(tr), om


@pytest.mark.parametrize("d,S", [(2, 5), (2, 8), (3, 6)])
def test_residual_and_jacobian_match_oracle(d, S):
    s, tr, tb, om = _case(d, S)
    z0 = 0.2 * np.random.default_rng(3).normal(size=(4, tb.Stilde))
    ref = oht.evaluate(s, tr, om, z0, sens=True, tables=tb)
    ctx = fse().fse_init_torus(s, tr)
    R, rn, J = fse().fse_hypertime_residual_jacobian(ctx, om[None], z0[None], want_J=True)
    assert rel(R[0].cpu().numpy(), ref["R"]) < RTOL
    assert abs(rn[0] - np.linalg.norm(ref["R"])) < RTOL * np.linalg.norm(ref["R"])
    assert rel(J[0].cpu().numpy(), oht.jacobian(ref)) < RTOL


def test_c1_residual_jacobian_and_gamma_identity():
    """10-DOF cantilever at full size (320 hyper-time unknowns): residual and Jacobian vs the
    oracle; at zbar(0) = Gamma Z(0) the residual is Gamma times the multi-frequency one."""
    wl = workload("C1")
    tb = osh.TorusTables(wl.torus)
    Z0 = wl.initial_iterate(tb.table)
    z0 = Z0 @ tb.G.T
    ref = oht.evaluate(wl.system, wl.torus, wl.omega, z0, sens=True, tables=tb)
    ctx = fse().fse_init_torus(wl.system, wl.torus)
    R, rn, J = fse().fse_hypertime_residual_jacobian(ctx, wl.omega[None], z0[None], want_J=True)
    assert rel(R[0].cpu().numpy(), ref["R"]) < RTOL
    assert rel(J[0].cpu().numpy(), oht.jacobian(ref)) < RTOL
    Rm, _, _ = fse().fse_shooting_residual_jacobian(ctx, wl.omega[None], Z0[None])
    assert rel(R[0].cpu().numpy(), Rm[0].cpu().numpy() @ tb.G.T) < RTOL


def test_newton_reaches_the_sampled_multifrequency_torus():
    import torch
    s, tr, tb, om = _case(2, 8)
    s.F *= 0.5
    zo, ho = oht.solve(s, tr, om, np.zeros((4, tb.Stilde)), tol_R=1e-13, tables=tb)
    ctx = fse().fse_init_torus(s, tr)
    z = torch.zeros((4, tb.Stilde), dtype=torch.float64, device="cuda")
    hist = []
    for _ in range(12):
        rn = fse().fse_hypertime_newton_step(ctx, om, z)
        hist.append(rn)
        if rn < 1e-13:
            break
    log(f"hyper-time Newton ||R|| history {['%.1e' % h for h in hist]}")
    assert hist[-1] < 1e-12
    zg = z.cpu().numpy()
    assert rel(zg, zo) < 1e-9
    Zm = torch.zeros((4, tb.U), dtype=torch.float64, device="cuda")
    fse().fse_newton_solve(ctx, om, Zm, tol=1e-13, maxit=20)
    assert rel(zg, Zm.cpu().numpy() @ tb.G.T) < 1e-9


@pytest.mark.parametrize("S", [5, 7])
def test_unknown_frequency_bordered_step(S):
    """d = 2, e = 1 (S~ = U~ and S~ > U~): the bordered hyper-time step equals the oracle's,
    samples and omega_2 within 1e-10 relative."""
    import torch
    from oracle import hypertime as oht
    s = tiny_system(n=2, seed=8, cubic=1.0, quad=0.3, e=1)
    tr = Torus(d=2, e=1, K=[np.arange(1, 3)], S=[S], S1=20)
    tb = osh.TorusTables(tr)
    om = np.array([1.05, 1.05 * (1 + 5 ** 0.5) / 2])
    Z0 = 0.2 * np.random.default_rng(2).normal(size=(4, tb.U))
    zb0 = Z0 @ tb.G.T
    zb1, om1, r0 = oht.newton_step(s, tr, om, zb0, tables=tb)
    ctx = fse().fse_init_torus(s, tr)
    zg = torch.tensor(zb0, dtype=torch.float64, device="cuda")
    omg = om.copy()
    rn = fse().fse_hypertime_newton_step(ctx, omg, zg)
    print(f"bordered hyper-time S={S}: omega_2 {omg[1]:.14f} (oracle {om1[1]:.14f})", flush=True)
    assert abs(rn - r0) < 1e-12 * r0
    assert np.linalg.norm(zg.cpu().numpy() - zb1) < 1e-10 * np.linalg.norm(zb1)
    assert abs(omg[1] - om1[1]) < 1e-10 * abs(om1[1])

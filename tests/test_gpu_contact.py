"""GPU trajectories with unilateral penalty contacts (a nonsmooth f_nl, the paper's third
recommendation) against the oracle.

Bar: states, sensitivities, residual, Jacobian and dR/dp within 1e-10 normwise relative
of the oracle (both sides decide in FP64 whether a contact is closed), also for the C1
cantilever against a stop at full size; Newton solves of the impact oscillator (d = 1 and
d = 2) reach ||R|| < 1e-8 and equal the oracle's tori within 1e-8; Lyapunov exponents
within 1e-6.
"""
import dataclasses

import numpy as np
import pytest

from _velocity_systems import impact_oscillator, with_contacts
from fse_inputs import Torus, tiny_system, workload
from oracle import continuation as ocont
from oracle import lyapunov as oly
from oracle import shooting as osh

pytestmark = pytest.mark.gpu
RTOL = 1e-10
GOLDEN = (1 + 5 ** 0.5) / 2


def fse():
    import paper_2508_06302_amd as m
    return m


def rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def log(msg):
    print(msg, flush=True)


def _case(d, e, beta=0.25, gamma=0.5, n=3, seed=2):
    s0 = tiny_system(n=n, seed=seed, cubic=1.0, quad=0.3, e=e)
    s = with_contacts(s0, [0, n - 1, 1], [1, -1, 1], [0.05, 0.02, 0.0], [5.0, 3.0, 2.0])
    om = np.array([1.1, 1.1 * GOLDEN, 1.1 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=e, K=[np.arange(1, 4)] * (d - 1), S=[8] * (d - 1), S1=64, beta=beta, gamma=gamma)
    tb = osh.TorusTables(tr)
    Z0 = 0.2 * np.random.default_rng(seed).normal(size=(2 * n, tb.U))
    return s0, s, tr, tb, om, Z0


@pytest.mark.parametrize("beta,gamma", [(0.25, 0.5), (0.3025, 0.6)])
@pytest.mark.parametrize("n", [3, 12])
def test_states_sensitivities_residual_and_jacobian(n, beta, gamma):
    s0, s, tr, tb, om, Z0 = _case(2, 2, beta, gamma, n=n)
    log(f"contacts n={n} beta={beta} gamma={gamma}")
    ref = osh.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    assert rel(osh.evaluate(s0, tr, om, Z0, tables=tb)["zbarT"], ref["zbarT"]) > 1e-4
    ctx = fse().fse_init_torus(s, tr)
    zT, phi = fse().fse_integrate_batch(ctx, om[None], Z0[None], want_phi=True)
    assert rel(zT[0].cpu().numpy(), ref["zbarT"]) < RTOL
    assert rel(phi[0].cpu().numpy(), ref["Phi"]) < RTOL
    R, rn, J = fse().fse_shooting_residual_jacobian(ctx, om[None], Z0[None], want_J=True)
    assert rel(R[0].cpu().numpy(), ref["R"]) < RTOL
    assert rel(J[0].cpu().numpy(), osh.jacobian(ref)) < RTOL
    # removing the contacts gives the smooth system's result
    fse().fse_set_contacts(ctx, [], [], [], [])
    zT0, _ = fse().fse_integrate_batch(ctx, om[None], Z0[None])
    assert rel(zT0[0].cpu().numpy(), osh.evaluate(s0, tr, om, Z0, tables=tb)["zbarT"]) < RTOL


@pytest.mark.parametrize("d,e", [(2, 2), (3, 2)])
def test_residual_dp(d, e):
    s0, s, tr, tb, om, Z0 = _case(d, e)
    ref = osh.evaluate(s, tr, om, Z0, omega_sens=True, tables=tb)
    dref = ocont.residual_dp(ref, om, e)
    ctx = fse().fse_init_torus(s, tr)
    R, dRdp = fse().fse_residual_dp(ctx, om[None], Z0[None])
    assert rel(R[0].cpu().numpy(), ref["R"]) < RTOL
    err = rel(dRdp[0].cpu().numpy().ravel(), dref)
    log(f"contacts dR/dp d={d} e={e}: rel err {err:.2e}")
    assert err < RTOL


def test_impact_oscillator_d1_newton_and_lyapunov():
    import torch
    s = impact_oscillator()
    tr = Torus(d=1, e=1, K=[], S=[], S1=256)
    om = np.array([1.3])
    tb = osh.TorusTables(tr)
    Z0 = np.zeros((2, tb.U))
    ctx = fse().fse_init_torus(s, tr)
    Zg = torch.tensor(Z0, dtype=torch.float64, device="cuda")
    it, rn = fse().fse_newton_solve(ctx, om, Zg, tol=1e-10, maxit=25)
    log(f"impact oscillator d=1: {it} Newton iterations, ||R|| {rn:.3e}")
    assert rn < 1e-8
    Zo, _, hist = osh.solve(s, tr, om, Z0, tol_R=1e-10, max_newton=25, tables=tb)
    assert rel(Zg.cpu().numpy(), Zo) < 1e-8
    sg = fse().fse_lyapunov(ctx, om, Zo, N_Ly=200)
    res = osh.evaluate(s, tr, om, Zo, sens=True, tables=tb)
    so = oly.exponents(res["Phi"], om, tb, N_Ly=200)[0]
    assert np.max(np.abs(sg - so)) < 1e-6 and np.max(so) < 0


def test_impact_oscillator_d2_newton_history_and_lyapunov():
    """Two-frequency forcing of the impact oscillator (a stiff stop, kc = 4): plain Newton steps
    on the GPU from the contact-free linear torus follow the oracle's iterates (seven steps,
    residual histories within 1e-6 relative), land on its torus, and give its Lyapunov exponents."""
    import torch
    s = dataclasses.replace(impact_oscillator(kc=4.0), F=np.array([[0.6], [0.25]]))
    s0 = dataclasses.replace(s, con_k=np.zeros(1))
    tr = Torus(d=2, e=2, K=[np.arange(1, 8)], S=[16], S1=128)
    om = np.array([0.7, 0.7 * GOLDEN])
    tb = osh.TorusTables(tr)
    Zl, _, _ = osh.solve(s0, tr, om, np.zeros((2, tb.U)), tol_R=1e-12, tables=tb)
    Zo, _, hist = osh.solve(s, tr, om, Zl, tol_R=1e-10, max_newton=25, tables=tb)
    ctx = fse().fse_init_torus(s, tr)
    Zg = torch.tensor(Zl, dtype=torch.float64, device="cuda")
    hg = [fse().fse_newton_step(ctx, om, Zg) for _ in range(len(hist) - 1)]
    R, rn, _ = fse().fse_shooting_residual_jacobian(ctx, om[None], Zg[None])
    log(f"impact oscillator d=2: oracle {['%.2e' % x for x in hist]} GPU {['%.2e' % x for x in hg]} "
        f"final {float(rn[0]):.2e}")
    assert np.allclose(hg, hist[:-1], rtol=1e-6)
    assert float(rn[0]) < 1e-8
    assert rel(Zg.cpu().numpy(), Zo) < 1e-8
    sg = fse().fse_lyapunov(ctx, om, Zo, N_Ly=200)
    res = osh.evaluate(s, tr, om, Zo, sens=True, tables=tb)
    so = oly.exponents(res["Phi"], om, tb, N_Ly=200)[0]
    log(f"Lyapunov GPU {sg} oracle {so}")
    assert np.max(np.abs(sg - so)) < 1e-6 and np.max(so) < 0


def test_c1_cantilever_against_a_stop_full_size():
    """C1 (n = 10, 16 trajectories of 256 steps) with a soft stop (2e3 N/m) 1e-4 m above the
    tip's rest position: residual and Jacobian at the initial iterate within 1e-10 of the
    oracle.  A stop a hundred times stiffer makes this map so sensitive that the oracle's own
    result moves by 3e-11 (R) and 2e-9 (J) between step tolerances 1e-12 and 1e-15, so no
    implementation with another rounding order could be held to 1e-10 there."""
    wl = workload("C1")
    tip = int(wl.system.t3_idx[0, 0])
    s = with_contacts(wl.system, [tip], [1], [1.0e-4], [2.0e3])
    tr = wl.torus
    tb = osh.TorusTables(tr)
    Z0 = wl.initial_iterate(tb.table)
    ref = osh.evaluate(s, tr, wl.omega, Z0, sens=True, tables=tb)
    free = osh.evaluate(wl.system, tr, wl.omega, Z0, tables=tb)
    assert rel(free["R"], ref["R"]) > 1e-3
    ctx = fse().fse_init_torus(s, tr)
    R, rn, J = fse().fse_shooting_residual_jacobian(ctx, wl.omega[None], Z0[None], want_J=True)
    eR, eJ = rel(R[0].cpu().numpy(), ref["R"]), rel(J[0].cpu().numpy(), osh.jacobian(ref))
    log(f"C1 with a tip stop: R rel err {eR:.2e}, J rel err {eJ:.2e}")
    assert eR < RTOL and eJ < RTOL


def test_invalid_contacts_and_mixed_precision():
    s0, s, tr, tb, om, Z0 = _case(2, 2)
    ctx = fse().fse_init_torus(s0, tr)
    for args in [([3], [1], [0.0], [1.0]), ([-1], [1], [0.0], [1.0]), ([0], [0], [0.0], [1.0]),
                 ([0], [1], [float("nan")], [1.0]), ([0], [1], [0.0], [-1.0]), ([0], [1], [0.0], [float("inf")])]:
        with pytest.raises(fse().FseError, match="FSE_E_INVAL"):
            fse().fse_set_contacts(ctx, *args)
    cm = fse().fse_init_torus(s, tr, precision=fse().FSE_PREC_MIXED_FP32)
    with pytest.raises(fse().FseError, match="FSE_E_UNSUPPORTED"):
        fse().fse_integrate_batch(cm, om[None], Z0[None], want_phi=True)


def test_impact_oscillator_arclength_matches_oracle():
    """Pseudo-arclength continuation in omega_1 of the impact oscillator's orbit (d = 1): eight
    points on the GPU equal the oracle's path."""
    s = impact_oscillator()
    tr = Torus(d=1, e=1, K=[], S=[], S1=256)
    tb = osh.TorusTables(tr)
    om0 = np.array([1.3])
    Z0, _, _ = osh.solve(s, tr, om0, np.zeros((2, 1)), tol_R=1e-12, tables=tb)
    path = ocont.arclength(s, tr, om0, Z0, 0.3, 8, tables=tb, tol_R=1e-11)
    ctx = fse().fse_init_torus(s, tr)
    Z, om, steps, it, rn = fse().fse_arclength(ctx, om0, Z0, 0.3, 8, tol=1e-11, maxit=8)
    log(f"impact oscillator branch: omega {np.round(om[:, 0], 5).tolist()}, corrections {it.tolist()}")
    assert np.all(rn < 1e-11)
    for j, p in enumerate(path):
        assert abs(om[j][0] - p["omega"][0]) < 1e-9 * p["omega"][0], (j, om[j], p["omega"])
        assert rel(Z[j].cpu().numpy(), p["Z"]) < 1e-8
        assert steps[j] == p["s"]

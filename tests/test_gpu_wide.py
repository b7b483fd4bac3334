"""GPU parity of the wide-band trajectory path (lumped mass, half bandwidth above 16): the
batched shared-S chord for the states and the banded LDL^T + matrix-core block sweeps for the
sensitivities (App. E, Eqs. E4-E9), through the C-ABI, against the FP64 oracle.

Bar: states, sensitivities, residuals and Jacobians within 1e-10 normwise relative of the oracle,
and every entry within 1e-9 of itself plus the largest entry of its block (sensitivities of the
full shell, products of 1024 step matrices: 1e-9 normwise).  The mixed mode keeps FP32
sensitivities: 1e-4.  The full-size shell is compared with stored oracle values
(tests/golden/c3_sampled.txt, written by tests/golden/make_c3_golden.py).
"""
import os

import numpy as np
import pytest

from _parity import elementwise, rel
from fse_inputs import Torus, tiny_system, workload
from fse_inputs.systems import banded_lumped_system, synthetic_shell
from oracle import shooting as osh

pytestmark = pytest.mark.gpu
GOLDEN = (1 + 5 ** 0.5) / 2
RTOL = 1e-10
HERE = os.path.dirname(os.path.abspath(__file__))


def fse():
    import paper_2508_06302_amd as m
    return m


def log(msg):
    print(msg, flush=True)


def lumped(s):
    import dataclasses
    return dataclasses.replace(s, M=np.diag(np.diag(s.M)))


def _check_eval(s, tr, om, Z0, prec=0, B=1, tol=RTOL, etol=1e-9):
    tb = osh.TorusTables(tr)
    n = s.n
    oms = np.stack([om * (1 + 0.02 * b) for b in range(B)])
    Zs = np.stack([Z0 * (1 - 0.3 * b) for b in range(B)])
    ctx = fse().fse_init_torus(s, tr, max_batch=B, precision=prec)
    zT, phi = fse().fse_integrate_batch(ctx, oms, Zs, want_phi=True)
    R, rn, J = fse().fse_shooting_residual_jacobian(ctx, oms, Zs, want_J=True)
    for b in range(B):
        ref = osh.evaluate(s, tr, oms[b], Zs[b], sens=True, tables=tb)
        z = zT[b].cpu().numpy()
        p = phi[b].cpu().numpy()
        assert rel(z, ref["zbarT"]) < RTOL
        elementwise(z, ref["zbarT"], 1e-9, n)
        assert rel(p, ref["Phi"]) < tol, rel(p, ref["Phi"])
        elementwise(p, ref["Phi"], etol, n)
        assert rel(R[b].cpu().numpy(), ref["R"]) < RTOL
        assert rel(J[b].cpu().numpy(), osh.jacobian(ref)) < tol
    return ctx


@pytest.mark.parametrize("d", [2, 3])
def test_wide_tiny_lumped(d, monkeypatch):
    """n = 3 (one ragged 16-row block, six of 16 columns used), forced onto the wide path."""
    monkeypatch.setenv("FSE_KERNELS", "wide")
    s = lumped(tiny_system(n=3, seed=2, cubic=1.0, quad=0.3, e=d))
    om = np.array([0.8, 0.8 * GOLDEN, 0.8 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=d, K=[np.arange(1, 4)] * (d - 1), S=[8] * (d - 1), S1=64)
    tb = osh.TorusTables(tr)
    Z0 = 0.2 * np.random.default_rng(2).normal(size=(6, tb.U))
    log(f"wide tiny d={d}")
    _check_eval(s, tr, om, Z0)


def test_wide_ragged_band_two_points(monkeypatch):
    """n = 37, half band 20 (two 16-row blocks below the diagonal, three row blocks, the last
    one ragged), 74 sensitivity columns (ragged tile), two continuation points in one call."""
    s = banded_lumped_system(n=37, bw=20, seed=3)
    tr = Torus(d=2, e=2, K=[np.arange(1, 4)], S=[8], S1=48)
    tb = osh.TorusTables(tr)
    om = np.array([1.1, 1.1 * GOLDEN])
    Z0 = 0.3 * np.random.default_rng(4).normal(size=(2 * s.n, tb.U))
    log("wide ragged band, B = 2")
    ctx = _check_eval(s, tr, om, Z0, B=2)
    mx, tot = fse().fse_step_stats(ctx)
    log(f"chord iterations: max {mx}, total {tot}")
    assert 1 <= mx <= 30


def test_wide_small_shell_newton(monkeypatch):
    """240-DOF shell (4 x 8 mesh, half band 35): evaluation parity, then GPU Newton-Krylov
    (matrix-free J v from the wide path's Phi) to the torus the oracle's dense Newton reaches."""
    s = synthetic_shell(NH=4, NL=8)
    tr = Torus(d=2, e=2, K=[np.arange(1, 3)], S=[6], S1=40)
    tb = osh.TorusTables(tr)
    w1 = 2 * np.pi * 100.0 * 0.9
    om = np.array([w1, w1 / 2 ** 0.5])
    from fse_inputs.systems import _linear_harmonics, place_harmonics
    Z0 = place_harmonics(tb.table, _linear_harmonics(s, om, [(0,), (1,)]), s.n, tb.U)
    log("wide 240-DOF shell evaluation")
    _check_eval(s, tr, om, Z0)
    import torch
    ctx = fse().fse_init_torus(s, tr)
    Zg = torch.tensor(Z0, dtype=torch.float64, device="cuda")
    hist = []
    for _ in range(6):
        rn, its, _ = fse().fse_newton_krylov_step(ctx, om, Zg, rtol=1e-12, restart=40, maxit=400)
        hist.append(rn)
        if rn < 1e-10:
            break
    log(f"GPU Newton-Krylov residuals {hist}")
    Zo, _, ho = osh.solve(s, tr, om, Z0, tol_R=1e-10, tables=tb)
    Zgpu = Zg.cpu().numpy()
    assert np.linalg.norm(osh.evaluate(s, tr, om, Zgpu, tables=tb)["R"]) < 1e-8
    assert rel(Zgpu, Zo) < 1e-8


def test_wide_mixed_fp32_sensitivities(monkeypatch):
    """Mixed mode on the wide path: FP32 factor, FP32 matrix-core sweeps and FP32 P1/P2 storage;
    states stay FP64 and exact, the sensitivities within 1e-4 of the FP64 oracle."""
    s = banded_lumped_system(n=37, bw=20, seed=3)
    tr = Torus(d=2, e=2, K=[np.arange(1, 4)], S=[8], S1=48)
    tb = osh.TorusTables(tr)
    om = np.array([1.1, 1.1 * GOLDEN])
    Z0 = 0.3 * np.random.default_rng(4).normal(size=(2 * s.n, tb.U))
    ref = osh.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    ctx = fse().fse_init_torus(s, tr, precision=fse().FSE_PREC_MIXED_FP32)
    zT, phi = fse().fse_integrate_batch(ctx, om[None], Z0[None], want_phi=True)
    assert rel(zT[0].cpu().numpy(), ref["zbarT"]) < RTOL
    err = rel(phi[0].cpu().numpy(), ref["Phi"])
    log(f"mixed Phi rel err {err:.2e}")
    assert err < 1e-4


def _golden_c3():
    path = os.path.join(HERE, "golden", "c3_sampled.txt")
    lines = [l for l in open(path) if not l.startswith("#")]
    cols_line = [l for l in open(path) if l.startswith("# trajectories")][0]
    cols = [int(x) for x in cols_line.split("columns")[1].split()]
    out, i = {}, 0
    while i < len(lines):
        _, s, _its = lines[i].split()
        rows = np.array([[float(x) for x in l.split()] for l in lines[i + 1:i + 1 + 3744]])
        out[int(s)] = (rows[:, 0], rows[:, 1:])
        i += 1 + 3744
    return out, cols


def _c3_state_tol():
    """Ten times the measured floating-point conditioning of the shell's one-period map: a relative
    1e-15 change of z(0), or one ulp of omega_1, moves the oracle's own z(2 pi) by the amounts in
    tests/golden/c3_sensitivity.txt (written by make_c3_sensitivity.py); two correct FP64
    implementations that round differently at every step cannot be held closer than that."""
    vals = [float(l.split()[1]) for l in open(os.path.join(HERE, "golden", "c3_sensitivity.txt"))
            if not l.startswith("#")]
    return max(RTOL, 10.0 * max(vals))


def _fp32_phi_bar(wl):
    """A priori bound on the relative error of FP32 sensitivities over one period: the FP32
    banded LDL^T solve of an SPD step matrix errs by about u32 kappa_s per step, with kappa_s the
    2-norm condition number of the diagonally scaled step matrix (the unscaled one, 6.8e3 on the
    shell, reflects only the spread of the lumped masses); summed linearly over the S1 steps, with
    a factor 4 for the two triangular solves and the two recursion updates of each step."""
    h = 2 * np.pi / wl.torus.S1                     # average acceleration: c0 = 4 / h^2, c2 = 2 / h
    w1, sysm = wl.omega[0], wl.system
    S = w1 ** 2 * (4 / h ** 2) * sysm.M + w1 * (2 / h) * sysm.D + sysm.K
    dinv = 1.0 / np.sqrt(np.diag(S))
    ev = np.linalg.eigvalsh(S * dinv[:, None] * dinv[None, :])
    return 4.0 * wl.torus.S1 * 2.0 ** -24 * ev[-1] / ev[0]


@pytest.mark.parametrize("prec", [0, 1])
def test_c3_full_size_sampled(prec):
    """The 1872-DOF shell at full size (128 trajectories, S1 = 1024, all 3744 sensitivity
    columns): states and sampled sensitivity columns of three trajectories against the oracle
    (stored values).  States within the measured conditioning bar of _c3_state_tol (5.2e-10),
    sensitivity columns 1e-9 (FP64) or the a priori FP32 bound of _fp32_phi_bar (mixed, 9.8e-4)."""
    import torch
    gold, cols = _golden_c3()
    stol = _c3_state_tol()
    wl = workload("C3")
    ctx = fse().fse_init_torus(wl.system, wl.torus, precision=prec)
    U, St, bw, kt = fse().fse_get_layout(ctx)
    Z0 = wl.initial_iterate(kt)
    log(f"C3 full size, precision {prec}: integrate with sensitivities")
    zT, phi = fse().fse_integrate_batch(ctx, wl.omega[None], Z0[None], want_phi=True)
    tm = fse().fse_last_timing(ctx)
    log(f"C3 timing {tm}")
    n = wl.system.n
    ptol = 1e-9 if prec == 0 else _fp32_phi_bar(wl)
    log(f"sensitivity bar {ptol:.2e}")
    for s, (zg, pg) in gold.items():
        z = zT[0, :, s].cpu().numpy()
        p = phi[0, s][:, cols].cpu().numpy()
        log(f"trajectory {s}: state {rel(z, zg):.2e}, Phi columns {rel(p, pg):.2e}")
        assert rel(z, zg) < stol
        elementwise(z, zg, 4 * stol, n)
        assert rel(p, pg) < ptol
        if prec == 0:
            for c in range(len(cols)):
                elementwise(p[:, c], pg[:, c], 1e-8, n)
    del phi
    torch.cuda.empty_cache()

"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Bar: bit-exact for the harmonic table; normwise relative <= 1e-10 for FP64
states, sensitivities and residuals; ||R|| < 1e-8 on converged tori with the
oracle re-evaluating R at the GPU's Z(0); Lyapunov exponents within 1e-6.
"""
import math

import numpy as np
import pytest

from fse_inputs import Torus, tiny_system, workload
from fse_inputs.systems import System
from oracle import lyapunov as olyap
from oracle import shooting as osh
from oracle import torus as otor

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


@pytest.mark.parametrize("K,S", [([np.arange(1, 6)], [16]), ([np.arange(1, 9)] * 2, [32, 32]),
                                 ([[1, 3], [1, 2], [2]], [7, 5, 5])])
def test_layout_bit_exact(K, S):
    d = len(K) + 1
    s = tiny_system(n=2, seed=1, e=d)
    tr = Torus(d=d, e=d, K=K, S=S, S1=8)
    ctx = fse().fse_init_torus(s, tr)
    U, St, bw, kt = fse().fse_get_layout(ctx)
    ref = otor.harmonic_table(K)
    assert U == otor.n_coefficients(K) and St == int(np.prod(S))
    assert np.array_equal(kt, ref)


def _tiny_case(d=2, n=3, S1=64, seed=2):
    s = tiny_system(n=n, seed=seed, cubic=1.0, quad=0.3, e=d)
    om = np.array([0.8, 0.8 * GOLDEN, 0.8 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=d, K=[np.arange(1, 4)] * (d - 1), S=[8] * (d - 1), S1=S1)
    tb = osh.TorusTables(tr)
    Z0 = 0.2 * np.random.default_rng(seed).normal(size=(2 * n, tb.U))
    return s, tr, tb, om, Z0


@pytest.mark.parametrize("kernels", ["fused", "generic"])
@pytest.mark.parametrize("d", [2, 3])
def test_integrate_state_and_sensitivities_tiny(d, kernels, monkeypatch):
    monkeypatch.setenv("FSE_KERNELS", kernels)
    s, tr, tb, om, Z0 = _tiny_case(d=d)
    log(f"tiny d={d} kernels={kernels}")
    ref = osh.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    ctx = fse().fse_init_torus(s, tr)
    zT, phi = fse().fse_integrate_batch(ctx, om[None], Z0[None], want_phi=True)
    assert rel(zT[0].cpu().numpy(), ref["zbarT"]) < RTOL
    assert rel(phi[0].cpu().numpy(), ref["Phi"]) < RTOL


def test_residual_and_jacobian_tiny():
    s, tr, tb, om, Z0 = _tiny_case()
    ref = osh.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    Jref = osh.jacobian(ref)
    ctx = fse().fse_init_torus(s, tr)
    R, rn, J = fse().fse_shooting_residual_jacobian(ctx, om[None], Z0[None], want_J=True)
    assert rel(R[0].cpu().numpy(), ref["R"]) < RTOL
    assert abs(rn[0] - np.linalg.norm(ref["R"])) < RTOL * np.linalg.norm(ref["R"])
    assert rel(J[0].cpu().numpy(), Jref) < RTOL


def test_batch_of_points_matches_single_calls():
    """B = 3 continuation points with different omega in one launch."""
    s, tr, tb, om, Z0 = _tiny_case()
    oms = np.stack([om, om * 1.01, om * 0.97])
    Zs = np.stack([Z0, 0.5 * Z0, -Z0])
    ctx = fse().fse_init_torus(s, tr, max_batch=3)
    zT, phi = fse().fse_integrate_batch(ctx, oms, Zs, want_phi=True)
    for b in range(3):
        ref = osh.evaluate(s, tr, oms[b], Zs[b], sens=True, tables=tb)
        assert rel(zT[b].cpu().numpy(), ref["zbarT"]) < RTOL
        assert rel(phi[b].cpu().numpy(), ref["Phi"]) < RTOL


def test_c1_full_newton_solve():
    """C1: GPU Newton to ||R|| < 1e-8 from the seeded start; the oracle re-evaluates R at
    the GPU's Z(0) and its own converged torus agrees."""
    wl = workload("C1")
    tb = osh.TorusTables(wl.torus)
    Z0 = wl.initial_iterate(tb.table)
    ctx = fse().fse_init_torus(wl.system, wl.torus)
    import torch
    Zg = torch.tensor(Z0, dtype=torch.float64, device="cuda")
    it, rn = fse().fse_newton_solve(ctx, wl.omega, Zg, tol=1e-8, maxit=10)
    log(f"C1 gpu newton iterations {it} |R| {rn:.3e}")
    assert rn < 1e-8
    Zgpu = Zg.cpu().numpy()
    ref = osh.evaluate(wl.system, wl.torus, wl.omega, Zgpu, tables=tb)
    assert np.linalg.norm(ref["R"]) < 1e-8
    Zo, _, hist = osh.solve(wl.system, wl.torus, wl.omega, Z0, tol_R=1e-10, tables=tb)
    assert rel(Zgpu, Zo) < 1e-8


@pytest.mark.parametrize("kernels", ["fused", "generic"])
def test_c1_integrate_all_trajectories(kernels, monkeypatch):
    monkeypatch.setenv("FSE_KERNELS", kernels)
    wl = workload("C1")
    tb = osh.TorusTables(wl.torus)
    Z0 = wl.initial_iterate(tb.table)
    ref = osh.evaluate(wl.system, wl.torus, wl.omega, Z0, sens=True, tables=tb)
    ctx = fse().fse_init_torus(wl.system, wl.torus)
    zT, phi = fse().fse_integrate_batch(ctx, wl.omega[None], Z0[None], want_phi=True)
    assert rel(zT[0].cpu().numpy(), ref["zbarT"]) < RTOL
    assert rel(phi[0].cpu().numpy(), ref["Phi"]) < RTOL


def test_c2_full_size_sampled_trajectories():
    """C2 at full size (147 DOF, 64 trajectories, S1 = 512): all trajectories on the
    GPU, three sampled ones (first, a middle one, the last) by the oracle."""
    wl = workload("C2")
    tb = osh.TorusTables(wl.torus)
    Z0 = wl.initial_iterate(tb.table)
    ctx = fse().fse_init_torus(wl.system, wl.torus)
    log("C2 gpu integrate with sensitivities")
    zT, phi = fse().fse_integrate_batch(ctx, wl.omega[None], Z0[None], want_phi=True)
    zT = zT[0].cpu().numpy()
    samples = [0, 37, 63]
    log("C2 oracle sampled trajectories")
    ref = osh.evaluate(wl.system, wl.torus, wl.omega, Z0, sens=True, tables=tb, samples=samples)
    for s in samples:
        assert rel(zT[:, s], ref["zbarT"][:, s]) < RTOL, s
        assert rel(phi[0, s].cpu().numpy(), ref["Phi"][s]) < 1e-9, s


def test_lyapunov_tiny_matches_oracle():
    s, tr, tb, om, Z0 = _tiny_case()
    ref = osh.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    Q0, _ = np.linalg.qr(np.random.default_rng(5).normal(size=(6, 6)))
    sig_o, _, _ = olyap.exponents(ref["Phi"], om, tb, N_Ly=200, Q0=Q0)
    ctx = fse().fse_init_torus(s, tr)
    sig_g = fse().fse_lyapunov(ctx, om, Z0, N_Ly=200, Q0=Q0)
    assert np.abs(sig_g - sig_o).max() < 1e-6


def test_d1_periodic_shooting():
    """d = 1 (classical shooting, Sec. 3.1): forced Duffing periodic orbit."""
    s = System("duffing", np.eye(1), np.array([[0.1]]), np.eye(1), np.zeros((0, 3), np.int32),
               np.zeros(0), np.array([[0, 0, 0, 0]], np.int32), np.array([0.5]), np.array([[0.4]]))
    tr = Torus(d=1, e=1, K=[], S=[], S1=128)
    om = np.array([0.7])
    tb = osh.TorusTables(tr)
    Zo, _, _ = osh.solve(s, tr, om, np.zeros((2, 1)), tol_R=1e-12, tables=tb)
    ctx = fse().fse_init_torus(s, tr)
    import torch
    Zg = torch.zeros((2, 1), dtype=torch.float64, device="cuda")
    it, rn = fse().fse_newton_solve(ctx, om, Zg, tol=1e-12, maxit=20)
    assert rn < 1e-12
    assert rel(Zg.cpu().numpy(), Zo) < 1e-10


def test_error_paths():
    m = fse()
    s, tr, tb, om, Z0 = _tiny_case()
    bad = Torus(d=2, e=2, K=[np.arange(1, 6)], S=[9], S1=16)     # S_2 < 2 H + 1
    with pytest.raises(m.FseError, match="FSE_E_INVAL"):
        m.fse_init_torus(s, bad)
    ctx = m.fse_init_torus(s, tr, max_batch=1)
    with pytest.raises(m.FseError, match="FSE_E_INVAL"):
        m.fse_integrate_batch(ctx, np.stack([om, om]), np.stack([Z0, Z0]))
    ctx1 = m.fse_init_torus(s, tr, step_maxit=1)
    with pytest.raises(m.FseError, match="FSE_E_NOCONV"):
        m.fse_integrate_batch(ctx1, om[None], Z0[None])
    ns = tiny_system(n=3, seed=2, e=2)
    ns.t2_idx = np.array([[0, 1, 2]], np.int32)                   # f_0 = q1 q2: not a gradient
    ns.t2_val = np.array([1.0])
    ns.t3_idx = np.zeros((0, 4), np.int32)
    ns.t3_val = np.zeros(0)
    with pytest.raises(m.FseError, match="FSE_E_UNSUPPORTED"):
        m.fse_init_torus(ns, tr)


def test_newton_step_ragged_lu():
    """One Newton step with N = 2 n U = 474 unknowns (7 full LU blocks and a ragged one)."""
    s = tiny_system(n=3, seed=4, cubic=1.0, quad=0.3, e=2)
    om = np.array([0.8, 0.8 * GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 40)], S=[96], S1=64)
    tb = osh.TorusTables(tr)
    Z0 = 0.1 * np.random.default_rng(7).normal(size=(6, tb.U)) / (1 + np.arange(tb.U))
    Zo, _, rn_o = osh.newton_step(s, tr, om, Z0, tables=tb)
    ctx = fse().fse_init_torus(s, tr)
    import torch
    Zg = torch.tensor(Z0, dtype=torch.float64, device="cuda")
    rn = fse().fse_newton_step(ctx, om, Zg)
    assert abs(rn - rn_o) < RTOL * rn_o
    assert rel(Zg.cpu().numpy() - Z0, Zo - Z0) < 1e-9


def test_c2_newton_step_solves_its_linearisation():
    """Full-size beam (N = 9114 unknowns): the LU runs its register-resident leaves of 8
    (panels of <= 5120 rows) and of 4 columns (<= 9216 rows).  The Newton update dZ must
    satisfy R + J dZ = 0 with the J and R of the same point (J applied on the host)."""
    import torch
    wl = workload("C2")
    ctx = fse().fse_init_torus(wl.system, wl.torus)
    U, St, bw, kt = fse().fse_get_layout(ctx)
    fse().fse_set_forcing(ctx, [0.3, 0.3])
    Z0 = torch.tensor(wl.initial_iterate(kt) * 0.3, dtype=torch.float64, device="cuda")
    R, rn, J = fse().fse_shooting_residual_jacobian(ctx, wl.omega[None], Z0[None], want_J=True)
    Rh = R[0].cpu().numpy().ravel()
    Jh = J[0].cpu().numpy()
    del J
    Zg = Z0.clone()
    rn2 = fse().fse_newton_step(ctx, wl.omega.copy(), Zg)
    assert abs(rn2 - rn[0]) <= 1e-14 * rn[0]
    dZ = (Zg - Z0).cpu().numpy().ravel()
    lin = np.linalg.norm(Rh + Jh @ dZ) / np.linalg.norm(Rh)
    log(f"C2 Newton step: ||R|| {rn[0]:.3e}, ||R + J dZ|| / ||R|| {lin:.2e}")
    assert lin < 1e-10


def test_secant_predict_matches_oracle():
    from oracle import learned as olearn
    s, tr, tb, om, Z0 = _tiny_case()
    rng = np.random.default_rng(11)
    Zp, Zc = rng.normal(size=Z0.shape), rng.normal(size=Z0.shape)
    pp, pc, pn = rng.normal(size=4), rng.normal(size=4), rng.normal(size=4)
    ctx = fse().fse_init_torus(s, tr)
    Zn = fse().fse_secant_predict(ctx, pp, pc, pn, Zp, Zc).cpu().numpy()
    assert rel(Zn, olearn.secant_predict(pp, pc, pn, Zp, Zc)) < 1e-14
    m = fse()
    with pytest.raises(m.FseError, match="FSE_E_INVAL"):
        m.fse_secant_predict(ctx, pc, pc, pn, Zp, Zc)


def test_forcing_amplitude_continuation_c1():
    """Natural-parameter continuation in the forcing amplitude (secant predictor):
    every point converged, re-evaluated by the oracle with the scaled loads."""
    import copy
    wl = workload("C1")
    tb = osh.TorusTables(wl.torus)
    Z0 = wl.initial_iterate(tb.table)
    amps = [0.25, 0.5, 0.75, 1.0]
    params = np.array([[*wl.omega, a, a] for a in amps])
    ctx = fse().fse_init_torus(wl.system, wl.torus)
    # ||R|| < 1e-12: the displacements are ~1e-4 m, so an absolute 1e-8 would leave the
    # solution defined only to ~1e-6 relative
    Z, it, rn = fse().fse_continuation(ctx, params, Z0, tol=1e-12, maxit=10)
    log(f"continuation iterations {it.tolist()} residuals {rn.tolist()}")
    assert np.all(it >= 0) and np.all(rn < 1e-12)
    ro = []
    for j, a in enumerate(amps):
        sj = copy.copy(wl.system)
        sj.F = wl.system.F * a
        ref = osh.evaluate(sj, wl.torus, wl.omega, Z[j].cpu().numpy(), tables=tb)
        fse().fse_set_forcing(ctx, [a, a])
        _, rg, _ = fse().fse_shooting_residual_jacobian(ctx, wl.omega[None], Z[j][None])
        ro.append((float(np.linalg.norm(ref["R"])), float(rg[0])))
    log(f"oracle / gpu residual at the gpu solutions: {ro}")
    assert all(r[0] < 1e-10 for r in ro)
    Zo, _, _ = osh.solve(wl.system, wl.torus, wl.omega, Z0, tol_R=1e-12, tables=tb)
    assert rel(Z[-1].cpu().numpy(), Zo) < 1e-8


def test_continuation_step_control_bisects():
    """A forcing step 0.1 -> 1.0 N that Newton cannot close in 4 iterations (the FP64
    oracle's full-step Newton needs 5 from the 0.1 N solution): the continuation halves the
    step, solves the inserted points, and returns the requested ones only.  Both results are
    re-evaluated by the oracle and the 1.0 N torus is the oracle's own solution."""
    import copy
    s = tiny_system(n=3, seed=2, cubic=1.0, quad=0.3, e=2)
    tr = Torus(d=2, e=2, K=[np.arange(1, 6)], S=[16], S1=64)
    tb = osh.TorusTables(tr)
    w = 0.45
    om = np.array([w, GOLDEN * w])
    amps = [0.1, 1.0]
    params = np.array([[*om, a, a] for a in amps])
    ctx = fse().fse_init_torus(s, tr)
    Z0 = np.zeros((6, ctx.U))
    Z, it, rn = fse().fse_continuation(ctx, params, Z0, tol=1e-12, maxit=4)
    log(f"step-controlled continuation: iterations {it.tolist()} residuals {rn.tolist()}")
    assert np.all(rn < 1e-12)
    # a single solve stops after maxit iterations: more at point 1 means inserted points
    assert it[1] > 4
    for j, a in enumerate(amps):
        sj = copy.copy(s)
        sj.F = s.F * a
        ref = osh.evaluate(sj, tr, om, Z[j].cpu().numpy(), tables=tb)
        assert np.linalg.norm(ref["R"]) < 1e-10, (a, np.linalg.norm(ref["R"]))
    s1 = copy.copy(s)
    s1.F = s.F * 0.1
    Zo1, _, _ = osh.solve(s1, tr, om, Z0, tol_R=1e-12, tables=tb)
    s1.F = s.F * 1.0
    Zo, _, h = osh.solve(s1, tr, om, Zo1, tol_R=1e-12, tables=tb)
    assert h[-1] < 1e-12
    assert rel(Z[1].cpu().numpy(), Zo) < 1e-8


def test_mixed_precision_sensitivities():
    """FP32 column state: states stay FP64-exact, Phi within 1e-4 normwise of the
    FP64 oracle (tiny and the 147-DOF beam, sampled trajectories)."""
    m = fse()
    s, tr, tb, om, Z0 = _tiny_case()
    ref = osh.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    ctx = m.fse_init_torus(s, tr, precision=m.FSE_PREC_MIXED_FP32)
    zT, phi = m.fse_integrate_batch(ctx, om[None], Z0[None], want_phi=True)
    assert rel(zT[0].cpu().numpy(), ref["zbarT"]) < RTOL
    e_tiny = rel(phi[0].cpu().numpy(), ref["Phi"])
    wl = workload("C2")
    tb2 = osh.TorusTables(wl.torus)
    Z2 = wl.initial_iterate(tb2.table)
    ctx2 = m.fse_init_torus(wl.system, wl.torus, precision=m.FSE_PREC_MIXED_FP32)
    zT2, phi2 = m.fse_integrate_batch(ctx2, wl.omega[None], Z2[None], want_phi=True)
    samples = [0, 63]
    ref2 = osh.evaluate(wl.system, wl.torus, wl.omega, Z2, sens=True, tables=tb2, samples=samples)
    e_c2 = max(rel(phi2[0, s_].cpu().numpy(), ref2["Phi"][s_]) for s_ in samples)
    log(f"mixed Phi error vs FP64 oracle: tiny {e_tiny:.2e}, 147-DOF beam {e_c2:.2e}")
    assert e_tiny < 1e-4 and e_c2 < 1e-4
    for s_ in samples:
        assert rel(zT2[0][:, s_].cpu().numpy(), ref2["zbarT"][:, s_]) < RTOL


def test_mixed_precision_newton_reaches_fp64_torus():
    """Newton with the FP32-sensitivity Jacobian still converges on the FP64 residual to
    the oracle's torus (C1, ||R|| < 1e-12)."""
    m = fse()
    wl = workload("C1")
    tb = osh.TorusTables(wl.torus)
    Z0 = wl.initial_iterate(tb.table)
    ctx = m.fse_init_torus(wl.system, wl.torus, precision=m.FSE_PREC_MIXED_FP32)
    import torch
    Zg = torch.tensor(Z0, dtype=torch.float64, device="cuda")
    it, rn = m.fse_newton_solve(ctx, wl.omega, Zg, tol=1e-12, maxit=20)
    log(f"mixed Newton: {it} iterations, |R| {rn:.2e}")
    assert rn < 1e-12
    Zo, _, _ = osh.solve(wl.system, wl.torus, wl.omega, Z0, tol_R=1e-12, tables=tb)
    assert rel(Zg.cpu().numpy(), Zo) < 1e-8


@pytest.mark.parametrize("d,e", [(2, 1), (3, 2)])
def test_unknown_frequency_bordered_newton_step(d, e):
    """d > e: dR/d omega_u (rotation term, Eq. 24 reading) and one bordered Newton step with
    the phase rows of Eq. (18), against the oracle from the same (Z0, omega)."""
    s = tiny_system(n=3, seed=6, cubic=1.0, quad=0.3, e=e)
    om = np.array([0.8, 0.8 * GOLDEN, 0.8 * 2 ** 0.5][:d])
    tr = Torus(d=d, e=e, K=[np.arange(1, 4)] * (d - 1), S=[8] * (d - 1), S1=64)
    tb = osh.TorusTables(tr)
    Z0 = 0.2 * np.random.default_rng(8).normal(size=(6, tb.U))
    res = osh.evaluate(s, tr, om, Z0, tables=tb)
    dref = osh.residual_domega(res, om, e, first=e + 1)
    ctx = fse().fse_init_torus(s, tr)
    R, dR = fse().fse_residual_domega(ctx, om[None], Z0[None])
    assert rel(R[0].cpu().numpy(), res["R"]) < RTOL
    assert rel(dR[0].cpu().numpy(), dref) < RTOL
    Zo, omo, rn_o = osh.newton_step(s, tr, om, Z0, tables=tb)
    import torch
    Zg = torch.tensor(Z0, dtype=torch.float64, device="cuda")
    omg = om.copy()
    rn = fse().fse_newton_step(ctx, omg, Zg)
    assert abs(rn - rn_o) < RTOL * rn_o
    assert rel(Zg.cpu().numpy() - Z0, Zo - Z0) < 1e-9
    assert np.abs((omg - om) - (omo - om)).max() < 1e-9 * np.abs(omo - om).max()
    m = fse()
    with pytest.raises(m.FseError, match="FSE_E_INVAL"):
        c2 = m.fse_init_torus(tiny_system(n=3, seed=6, e=d), Torus(d=d, e=d, K=tr.K, S=tr.S, S1=64))
        m.fse_residual_domega(c2, om[None], Z0[None])


def test_c4_three_frequency_batched_points_sampled():
    """Three-frequency beam (147 DOF, d = 3, 32 x 32 = 1024 trajectories, H = 8 x 8,
    S1 = 512) with two continuation points in one launch: every trajectory on the GPU,
    sampled trajectories of each point by the oracle."""
    wl = workload("C4")
    tb = osh.TorusTables(wl.torus)
    Z0 = wl.initial_iterate(tb.table)
    oms = np.stack([wl.omega, wl.omega * 1.0125])
    Zs = np.stack([Z0, Z0])
    ctx = fse().fse_init_torus(wl.system, wl.torus, max_batch=2)
    log("C4 gpu integrate, 2 points x 1024 trajectories with sensitivities")
    zT, phi = fse().fse_integrate_batch(ctx, oms, Zs, want_phi=True)
    for b, samples in ((0, [0, 517]), (1, [1023])):
        log(f"C4 oracle point {b} samples {samples}")
        ref = osh.evaluate(wl.system, wl.torus, oms[b], Zs[b], sens=True, tables=tb, samples=samples)
        for s_ in samples:
            assert rel(zT[b][:, s_].cpu().numpy(), ref["zbarT"][:, s_]) < RTOL, (b, s_)
            assert rel(phi[b, s_].cpu().numpy(), ref["Phi"][s_]) < 1e-9, (b, s_)


def test_autotuner_times_both_configs_and_they_agree(monkeypatch):
    """The fused kernel's column-wave count is tuned on the first launch with sensitivities;
    the candidate configurations compute bit-identical states and sensitivities."""
    m = fse()
    s, tr, tb, om, Z0 = _tiny_case(n=4)
    ctx = m.fse_init_torus(s, tr)
    zT, phi = m.fse_integrate_batch(ctx, om[None], Z0[None], want_phi=True)
    ncw, ms = m.fse_get_tuning(ctx)
    log(f"autotuner: {ncw} column waves; timed launches {ms.tolist()} ms")
    assert ncw in (1, 2) and ms.min() > 0 and ms[ncw - 1] == ms.min()
    outs = []
    for k in ("1", "2"):
        monkeypatch.setenv("FSE_FUSED_NCW", k)
        c = m.fse_init_torus(s, tr)
        outs.append(m.fse_integrate_batch(c, om[None], Z0[None], want_phi=True))
        assert m.fse_get_tuning(c)[0] == int(k)
    assert np.array_equal(outs[0][0].cpu().numpy(), outs[1][0].cpu().numpy())
    assert np.array_equal(outs[0][1].cpu().numpy(), outs[1][1].cpu().numpy())
    assert np.array_equal(phi.cpu().numpy(), outs[0][1].cpu().numpy())


@pytest.mark.parametrize("kernels", ["generic", "default"])
def test_wide_band_shell(kernels, monkeypatch):
    """A 360-DOF shell-like system (half bandwidth 47, 39k quadratic and 93k cubic force
    terms): by default it takes the wide-band path (lumped mass), with FSE_KERNELS=generic the
    generic kernels with their global-memory factor scratch; sampled trajectories against the
    oracle either way.  The FP32-sensitivity mode runs on the wide-band path (Phi within 1e-4)
    and is refused by the generic kernels (FSE_E_UNSUPPORTED)."""
    from fse_inputs.systems import synthetic_shell
    if kernels == "generic":
        monkeypatch.setenv("FSE_KERNELS", "generic")
    m = fse()
    s = synthetic_shell(NH=5, NL=10)
    w1 = 0.98 * 628.31853072
    om = np.array([w1, w1 / 2 ** 0.5])
    tr = Torus(d=2, e=2, K=[np.arange(1, 4)], S=[8], S1=64)
    tb = osh.TorusTables(tr)
    Z0 = 1e-3 * np.random.default_rng(21).normal(size=(2 * s.n, tb.U)) / (1 + np.arange(tb.U))
    ctx = m.fse_init_torus(s, tr)
    U, St, bw, kt = m.fse_get_layout(ctx)
    assert bw == 47
    log(f"wide-band shell ({kernels}): gpu integrate with sensitivities")
    zT, phi = m.fse_integrate_batch(ctx, om[None], Z0[None], want_phi=True)
    samples = [0, 5]
    log("wide-band shell: oracle samples")
    ref = osh.evaluate(s, tr, om, Z0, sens=True, tables=tb, samples=samples)
    for s_ in samples:
        assert rel(zT[0][:, s_].cpu().numpy(), ref["zbarT"][:, s_]) < RTOL, s_
        assert rel(phi[0, s_].cpu().numpy(), ref["Phi"][s_]) < 1e-9, s_
    cm = m.fse_init_torus(s, tr, precision=m.FSE_PREC_MIXED_FP32)
    if kernels == "generic":
        with pytest.raises(m.FseError, match="FSE_E_UNSUPPORTED"):
            m.fse_integrate_batch(cm, om[None], Z0[None], want_phi=True)
    else:
        _, phm = m.fse_integrate_batch(cm, om[None], Z0[None], want_phi=True)
        for s_ in samples:
            assert rel(phm[0, s_].cpu().numpy(), ref["Phi"][s_]) < 1e-4, s_

"""GPU Lyapunov exponents (App. F, Eqs. F1-F3) at finite-element sizes, through the C-ABI, against
the FP64 oracle: the 10-DOF cantilever with all 16 trajectories (oracle in the test), the 147-DOF
beam with 64 trajectories (294 x 294 one-period maps) and the three-frequency beam with 1024
trajectories (stored oracle values, tests/golden/lyapunov_c{2,4}.txt, written by
tests/golden/make_lyapunov_golden.py), and the phase-space-divergence invariant of a linearly
damped, resolved system.  Bar: every exponent within 1e-6 of the oracle's (absolute, 1/s)."""
import os

import numpy as np
import pytest

from _parity import rel
from fse_inputs import Torus, tiny_system, workload
from oracle import lyapunov as olyap
from oracle import shooting as osh

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = (1 + 5 ** 0.5) / 2


def fse():
    import paper_2508_06302_amd as m
    return m


def log(msg):
    print(msg, flush=True)


def _golden(name):
    """(exponents in QR order, their change when the start basis moves 1e-14 from the identity)."""
    rows = np.array([[float(x) for x in l.split()] for l in open(os.path.join(HERE, "golden", f"lyapunov_{name}.txt"))
                     if not l.startswith("#")])
    return rows[:, 0], rows[:, 1]


def test_lyapunov_c1_full_size():
    """C1: 20 x 20 maps, 16 trajectories, N_Ly = 1000; the sum also equals the mean log|det| of
    the interpolated maps (exact for any system)."""
    wl = workload("C1")
    tb = osh.TorusTables(wl.torus)
    Z0 = wl.initial_iterate(tb.table)
    ref = osh.evaluate(wl.system, wl.torus, wl.omega, Z0, sens=True, tables=tb)
    sig_o, _, acc = olyap.exponents(ref["Phi"], wl.omega, tb, N_Ly=1000)
    ctx = fse().fse_init_torus(wl.system, wl.torus)
    sig_g = fse().fse_lyapunov(ctx, wl.omega, Z0, N_Ly=1000)
    log(f"C1 max |dsigma| {np.abs(sig_g - sig_o).max():.2e}, sigma range {sig_o.min():.3e} .. {sig_o.max():.3e}")
    assert np.abs(sig_g - sig_o).max() < 1e-6
    T1 = 2 * np.pi / wl.omega[0]
    dets = []
    for i in range(1, 1001):
        phi = 2 * np.pi * (i - 1) * wl.omega[1:] / wl.omega[0]
        dets.append(np.linalg.slogdet(olyap.interpolated_transition(ref["Phi"], wl.omega, tb, phi))[1])
    assert abs(sig_g.sum() - np.mean(dets) / T1) < 1e-6 * max(1.0, abs(sig_g.sum()))


@pytest.mark.parametrize("name", ["c2", "c4"])
def test_lyapunov_beam_full_size(name):
    """The 147-DOF beam: 294 x 294 maps of 64 (d = 2) or 1024 (d = 3) trajectories, N_Ly = 1000,
    identity start basis, against the stored oracle exponents.  The spectrum spans 6 ... -233 1/s
    over a period of 0.157 s, so the product of the per-period maps spans far more than the FP64
    range: the strongly contracting exponents (and the members of clusters) are set by rounding on
    either side, and a 1e-14 change of the start basis alone moves the oracle's own values by the
    amounts stored with them (up to 0.26).  Held: every exponent that change moves by less than
    1e-8 (the FP64 sweep determines it) to 1e-6, among them the largest (the stability verdict of
    the torus); those it moves by less than 1e-5 to max(1e-6, 10 x that change).  The rest carry
    no per-exponent claim (the GPU's are finite)."""
    wl = workload(name.upper())
    ctx = fse().fse_init_torus(wl.system, wl.torus)
    U, St, bw, kt = fse().fse_get_layout(ctx)
    log(f"{name}: GPU Lyapunov exponents ({St} trajectories)")
    sig_g = fse().fse_lyapunov(ctx, wl.omega, wl.initial_iterate(kt), N_Ly=1000)
    sig_o, dsig = _golden(name)
    sens = np.abs(dsig)
    d = np.abs(sig_g - sig_o)
    strict, held = sens < 1e-8, sens < 1e-5
    log(f"{name}: largest exponent {sig_o.max():.6f}; {int(strict.sum())} exponents determined to 1e-8, "
        f"max |dsigma| there {d[strict].max():.2e}; {int(held.sum())} to 1e-5, max |dsigma|/max(1e-6, 10 sens) "
        f"there {np.max(d[held] / np.maximum(1e-6, 10 * sens[held])):.3f}; elsewhere max |dsigma| {d[~held].max():.2e}")
    assert sig_g.shape == sig_o.shape and np.all(np.isfinite(sig_g))
    assert strict.sum() >= 3 and strict[np.argmax(sig_o)]
    assert np.all(d[strict] < 1e-6)
    assert np.all(d[held] <= np.maximum(1e-6, 10 * sens[held]))
    assert abs(sig_g.max() - sig_o.max()) < 1e-6


def _trapezoidal_exponent_sum(s, omega1, S1):
    """Exact sum of the Lyapunov exponents of the average-acceleration map of a linear system.
    With beta = 1/4, gamma = 1/2 the Newmark step is the trapezoidal rule on x = [q; u], u = dq/dphi_1,
    x' = A x with A = [[0, I], [-M^-1 K / w1^2, -M^-1 D / w1]] in phi_1 (the velocity update averages
    the accelerations, and then the displacement update averages the velocities).  One step
    multiplies det by prod_i (1 + h l_i / 2) / (1 - h l_i / 2) over the eigenvalues l_i of A, so
    sum sigma = S1 sum_i log|(1 + h l_i / 2) / (1 - h l_i / 2)| / T1, T1 = 2 pi / w1; as h -> 0 this
    tends to tr(A) S1 h / T1 = -tr(M^-1 D)."""
    n = s.n
    MK = np.linalg.solve(s.M, s.K)
    MD = np.linalg.solve(s.M, s.D)
    A = np.block([[np.zeros((n, n)), np.eye(n)], [-MK / omega1 ** 2, -MD / omega1]])
    lam = np.linalg.eigvals(A)
    h = 2 * np.pi / S1
    per_step = np.sum(np.log(np.abs((1 + h * lam / 2) / (1 - h * lam / 2))))
    return S1 * per_step / (2 * np.pi / omega1)


def test_lyapunov_sum_is_phase_space_divergence():
    """Linear damping, all modes resolved (S1 = 512 per period): the exponents sum to the exact
    value of the discrete map (closed form of the trapezoidal rule, 1e-9 relative) and to
    log|det Psi| / T1 of the constant one-period map (1e-10), and that sum is -tr(M^-1 D) up to the
    rule's O(h^2) distortion (measured here, and at most half as large again)."""
    s = tiny_system(n=2, seed=4, nonlinear=False, zeta=0.05)
    om = np.array([0.9, 0.9 * GOLDEN])
    tr = Torus(d=2, e=2, K=[np.arange(1, 3)], S=[5], S1=512)
    tb = osh.TorusTables(tr)
    ctx = fse().fse_init_torus(s, tr)
    Z0 = np.zeros((4, tb.U))
    sig = fse().fse_lyapunov(ctx, om, Z0, N_Ly=200)
    target = -np.trace(np.linalg.solve(s.M, s.D))
    exact = _trapezoidal_exponent_sum(s, om[0], tr.S1)
    ref = osh.evaluate(s, tr, om, Z0, sens=True, tables=tb)
    Psi = olyap.transition_samples(ref["Phi"], om[0])[0]
    T1 = 2 * np.pi / om[0]
    log(f"sum {sig.sum():.12f}, discrete closed form {exact:.12f}, -tr(M^-1 D) {target:.12f}, "
        f"log|det Psi|/T1 {np.linalg.slogdet(Psi)[1] / T1:.12f}")
    assert abs(sig.sum() - np.linalg.slogdet(Psi)[1] / T1) < 1e-10
    assert abs(sig.sum() - exact) < 1e-9 * abs(exact)
    assert abs(sig.sum() - target) < 1.5 * abs(exact - target) + 1e-12


def _c4_state_tol():
    """Per point: max(1e-10, 10 x the measured floating-point conditioning of its sampled
    trajectory's one-period map), the relative change of the oracle's own zbar(2 pi) under a 1e-15
    relative change of zbar(0) or one ulp of omega_1 (tests/golden/c4_sensitivity.txt, written by
    make_c4_sensitivity.py).  At omega_1 = 39.5 rad/s one ulp of omega_1 alone moves it by 1.5e-10."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "c4_sensitivity.txt")) if not l.startswith("#")]
    return {int(r[0]): max(1e-10, 10.0 * max(float(r[2]), float(r[3]))) for r in rows}


def test_c4_eight_points_in_one_launch_sampled():
    """The three-frequency beam with 8 continuation points (omega_1 = 36.5 .. 40 rad/s) in one
    launch, 8 x 1024 trajectories with full sensitivities: for every point a sampled trajectory
    (a different one per point, first to last) against the oracle, states within the point's
    conditioning bar of _c4_state_tol (1e-10 where the map allows it) and sensitivities 1e-9
    normwise, and every point's residual against the GPU's single-point residual."""
    from _parity import elementwise
    m = fse()
    w1s = np.linspace(36.5, 40.0, 8)
    wls = [workload("C4", omega1=float(w)) for w in w1s]
    ctx = m.fse_init_torus(wls[0].system, wls[0].torus, max_batch=8)
    U, St, bw, kt = m.fse_get_layout(ctx)
    om = np.stack([w.omega for w in wls])
    Zs = np.stack([w.initial_iterate(kt) for w in wls])
    log("C4: 8 points, one launch with sensitivities")
    zT, phi = m.fse_integrate_batch(ctx, om, Zs, want_phi=True)
    tb = osh.TorusTables(wls[0].torus)
    n = wls[0].system.n
    stol = _c4_state_tol()
    for b, wl in enumerate(wls):
        s = (b * 146) % St
        ref = osh.evaluate(wl.system, wl.torus, wl.omega, Zs[b], sens=True, tables=tb, samples=[s])
        z = zT[b, :, s].cpu().numpy()
        p = phi[b, s].cpu().numpy()
        log(f"point {b} (omega_1 {w1s[b]:.2f}) trajectory {s}: state {rel(z, ref['zbarT'][:, s]):.2e}, "
            f"Phi {rel(p, ref['Phi'][s]):.2e} (state bar {stol[b]:.1e})")
        assert rel(z, ref["zbarT"][:, s]) < stol[b]
        elementwise(z, ref["zbarT"][:, s], 10 * stol[b], n)
        assert rel(p, ref["Phi"][s]) < 1e-9
    del phi
    R8, rn8, _ = m.fse_shooting_residual_jacobian(ctx, om, Zs)
    for b in (0, 7):
        R1, rn1, _ = m.fse_shooting_residual_jacobian(ctx, om[b:b + 1], Zs[b:b + 1])
        assert rel(R8[b].cpu().numpy(), R1[0].cpu().numpy()) < 1e-13

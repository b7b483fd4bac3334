"""The no-allocation entry point fse_jacobian_apply_noalloc (for callers that cannot allocate
device memory) against the allocating fse_jacobian_apply, through the C-ABI: two calls in a row
on the fixed per-GPU scratch, the second with a smaller problem, and the size limit."""
import numpy as np
import pytest

from fse_inputs import Torus, tiny_system, workload

pytestmark = pytest.mark.gpu


def fse():
    import paper_2508_06302_amd as m
    return m


def _case(ctx, wl_omega, Z0, seed):
    import torch
    m = fse()
    Zd = torch.tensor(Z0, dtype=torch.float64, device="cuda")
    m.fse_shooting_residual_matfree(ctx, wl_omega, Zd)
    v = torch.tensor(np.random.default_rng(seed).normal(size=Z0.shape), dtype=torch.float64, device="cuda")
    ref = m.fse_jacobian_apply(ctx, v)
    out = torch.full_like(v, float("nan"))
    m.fse_jacobian_apply_noalloc(ctx, v, out)
    return out.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_jv_matches_the_allocating_call_twice():
    m = fse()
    # first call: the 147-DOF beam (2n = 294, 64 trajectories)
    wl = workload("C2")
    ctx = m.fse_init_torus(wl.system, wl.torus)
    U, St, bw, kt = m.fse_get_layout(ctx)
    got, ref = _case(ctx, wl.omega, wl.initial_iterate(kt), 1)
    assert np.isfinite(got).all()
    assert np.array_equal(got, ref), float(np.abs(got - ref).max())
    # second call, smaller: a 3-DOF system with 8 trajectories, the scratch keeps the first call's
    # contents beyond what this call writes
    s = tiny_system(n=3, seed=2, cubic=1.0, quad=0.3, e=2)
    tr = Torus(d=2, e=2, K=[np.arange(1, 4)], S=[8], S1=64)
    c2 = m.fse_init_torus(s, tr)
    U2 = m.fse_get_layout(c2)[0]
    om = np.array([0.8, 0.8 * (1 + 5 ** 0.5) / 2])
    Z0 = 0.2 * np.random.default_rng(3).normal(size=(6, U2))
    got, ref = _case(c2, om, Z0, 4)
    assert np.array_equal(got, ref), float(np.abs(got - ref).max())
    # the first context again, after the smaller call
    got, ref = _case(ctx, wl.omega, wl.initial_iterate(kt), 5)
    assert np.array_equal(got, ref)


def test_noalloc_jv_refuses_problems_beyond_its_scratch():
    """2 x 2n x (max_batch S~) above 2^21 doubles: FSE_E_UNSUPPORTED (here the three-frequency beam
    sized for four continuation points: 2 x 294 x 4096)."""
    import torch
    m = fse()
    wl = workload("C4")
    ctx = m.fse_init_torus(wl.system, wl.torus, max_batch=4)
    U, St, bw, kt = m.fse_get_layout(ctx)
    Zd = torch.tensor(wl.initial_iterate(kt), dtype=torch.float64, device="cuda")
    m.fse_set_forcing(ctx, [0.1] * wl.system.e)
    m.fse_shooting_residual_matfree(ctx, wl.omega, 0.1 * Zd)
    out = torch.empty_like(Zd)
    with pytest.raises(m.FseError, match="FSE_E_UNSUPPORTED"):
        m.fse_jacobian_apply_noalloc(ctx, Zd, out)

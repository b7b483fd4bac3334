"""Pins of the oracle's predictors: secant, snapshot POD, MLP gradients."""
import numpy as np
import pytest

from oracle import learned


def test_secant_exact_on_affine_path():
    rng = np.random.default_rng(0)
    Z0, dZ = rng.normal(size=(5, 7)), rng.normal(size=(5, 7))
    p0, dp = rng.normal(size=3), rng.normal(size=3)
    path = lambda t: Z0 + t * dZ
    par = lambda t: p0 + t * dp
    Zp = learned.secant_predict(par(0.0), par(0.4), par(1.1), path(0.0), path(0.4))
    assert np.allclose(Zp, path(1.1), atol=1e-12)


def test_pod_matches_svd_and_is_orthonormal():
    rng = np.random.default_rng(1)
    N, m, r = 300, 40, 12
    X = rng.normal(size=(N, 6)) @ rng.normal(size=(6, m)) + 0.05 * rng.normal(size=(N, m))
    mean, B, sv = learned.pod_snapshots(X, r)
    assert np.allclose(B.T @ B, np.eye(r), atol=1e-10)
    Xc = X - X.mean(axis=1, keepdims=True)
    s_ref = np.linalg.svd(Xc, compute_uv=False)
    assert np.allclose(sv[:r], s_ref[:r], rtol=1e-9)
    rec = B @ (B.T @ Xc)
    err = np.linalg.norm(Xc - rec)
    assert np.isclose(err, np.sqrt(np.sum(s_ref[r:] ** 2)), rtol=1e-8)


@pytest.mark.parametrize("sizes", [(3, 8, 8, 4), (3, 256, 256, 64)])
def test_mlp_gradients_match_finite_differences(sizes):
    rng = np.random.default_rng(2)
    params = learned.mlp_init(sizes, seed=3)
    x = rng.normal(size=(5, sizes[0]))
    t = rng.normal(size=(5, sizes[-1]))
    g = learned.mlp_backward(params, x, t)
    h = 1e-6
    picks = [(0, 0, (1, 2)), (0, 1, (3,)), (1, 0, (2, 5)), (1, 1, (0,)), (2, 0, (1, 3)), (2, 1, (2,))]
    for li, pi, idx in picks:
        p = params[li][pi]
        old = p[idx]
        p[idx] = old + h
        lp = learned.mlp_loss(params, x, t)
        p[idx] = old - h
        lm = learned.mlp_loss(params, x, t)
        p[idx] = old
        fd = (lp - lm) / (2 * h)
        assert np.isclose(g[li][pi][idx], fd, rtol=1e-6, atol=1e-10), (li, pi, idx)


def test_gelu_reference_values():
    # GELU(x) = x Phi(x): Phi(1) = 0.841344746..., Phi(-1) = 0.158655253...
    assert np.isclose(learned.gelu(np.array(1.0)), 0.8413447460685429, rtol=1e-14)
    assert np.isclose(learned.gelu(np.array(-1.0)), -0.15865525393145707, rtol=1e-14)


def test_bf16_rounding_hand_worked_values():
    """bfloat16 keeps 8 significand bits: spacing 2^-7 on [1, 2)."""
    from oracle.learned import bf16_round
    cases = {1.0: 1.0, 1.0 + 2.0 ** -7: 1.0 + 2.0 ** -7,
             1.0 + 2.0 ** -8: 1.0,                       # tie, even stays
             1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,       # tie, odd rounds up
             1.0 + 2.0 ** -8 + 2.0 ** -12: 1.0 + 2.0 ** -7,
             -3.0: -3.0, 0.0: 0.0, 65536.0 + 128.0: 65536.0, 65536.0 + 384.0: 65536.0 + 512.0}
    for x, r in cases.items():
        assert bf16_round(x) == r, (x, bf16_round(x), r)
    v = np.random.default_rng(0).normal(size=1000)
    rv = bf16_round(v)
    assert np.all(np.abs(rv - v) <= 2.0 ** -8 * np.abs(v) * (1 + 1e-7))
    assert np.array_equal(bf16_round(rv), rv)


def _adamw_run(params, grads_seq, **kw):
    state = {}
    for g in grads_seq:
        params = learned.adamw_step(params, g, state, **kw)
    return params


def test_adamw_matches_torch_adamw():
    """The published AdamW rule (Adam moments with bias correction, weight decay decoupled from
    the gradient and scaled by the learning rate) as implemented by torch.optim.AdamW, in FP64."""
    import torch
    rng = np.random.default_rng(11)
    shapes = [(4, 3), (4,), (2, 4), (2,)]
    p0 = [rng.normal(size=sh) for sh in shapes]
    grads = [[rng.normal(size=sh) * (1 + 5 * k % 3) for sh in shapes] for k in range(25)]
    lr, wd = 3e-2, 5e-2
    params = [[p0[0].copy(), p0[1].copy()], [p0[2].copy(), p0[3].copy()]]
    out = _adamw_run(params, [[[g[0], g[1]], [g[2], g[3]]] for g in grads], lr=lr, wd=wd)
    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in p0]
    opt = torch.optim.AdamW(tp, lr=lr, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
    for g in grads:
        for t, gg in zip(tp, g):
            t.grad = torch.tensor(gg, dtype=torch.float64)
        opt.step()
    mine = [out[0][0], out[0][1], out[1][0], out[1][1]]
    for a, t in zip(mine, tp):
        assert np.allclose(a, t.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adamw_closed_forms():
    """Three consequences of the rule that a dropped bias correction, a wrong moment power or a
    decay coupled into the gradient would each break:
    (i) a constant gradient g moves every entry by lr g / (|g| + eps) per step, whatever |g|
        (m_t / (1 - b1^t) = g and v_t / (1 - b2^t) = g^2 exactly);
    (ii) with zero gradient the decoupled decay is geometric: p_T = (1 - lr wd)^T p_0;
    (iii) the first step is invariant under scaling the gradient (up to eps)."""
    lr = 1e-2
    p0 = np.array([0.7, -1.3, 2.0, 0.0])
    g = np.array([3.0, -0.02, 1e-3, -40.0])
    T = 17
    out = _adamw_run([[p0.copy()]], [[[g]]] * T, lr=lr, wd=0.0)[0][0]
    assert np.allclose(out, p0 - T * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)
    wd = 0.3
    out = _adamw_run([[p0.copy()]], [[[np.zeros(4)]]] * T, lr=lr, wd=wd)[0][0]
    assert np.allclose(out, (1 - lr * wd) ** T * p0, rtol=1e-14, atol=0)
    a = _adamw_run([[p0.copy()]], [[[g]]], lr=lr, wd=0.0, eps=0.0)[0][0]
    b = _adamw_run([[p0.copy()]], [[[1e4 * g]]], lr=lr, wd=0.0, eps=0.0)[0][0]
    assert np.allclose(a, b, rtol=0, atol=1e-15)
    assert np.allclose(a, p0 - lr * np.sign(g), rtol=0, atol=1e-15)

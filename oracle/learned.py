"""Continuation predictors (oracle; test infrastructure only).

The paper's continuation (App. C) predicts the next solution from the previous
ones; the secant predictor below is its zeroth-information form.  The learned
predictor is an MLP on POD coefficients of converged Z(0): it is not in the
paper, so every function here is pinned by identities rather than by paper
values:
  secant_predict  exact on affine paths (test)
  pod_snapshots   orthonormal basis; reconstruction error of the snapshots
                  equals the discarded singular values (test vs numpy SVD)
  mlp_*           forward in FP64; gradients vs central finite differences
  bf16_round      round-to-nearest-even to bfloat16 (8 significand bits), pinned by
                  hand-worked values; mlp_forward_bf16 is mlp_forward with every layer's
                  weights and inputs rounded to bfloat16 (the reduced-precision inference)
  adamw_step      the published AdamW rule (Adam with bias-corrected moments, weight decay
                  decoupled from the gradient and scaled by the learning rate), pinned by
                  torch.optim.AdamW in FP64 and by three closed forms: constant-gradient
                  steps of exactly lr g/(|g| + eps), geometric decay under zero gradient,
                  scale invariance of the first step
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def secant_predict(p_prev, p_cur, p_next, Z_prev, Z_cur):
    """Z^0_{j+1} = Z_j + tau (Z_j - Z_{j-1}), tau = (dp_next . dp) / |dp|^2."""
    dp = np.asarray(p_cur, float) - np.asarray(p_prev, float)
    dn = np.asarray(p_next, float) - np.asarray(p_cur, float)
    tau = float(dn @ dp) / float(dp @ dp)
    return Z_cur + tau * (Z_cur - Z_prev)


def pod_snapshots(X: np.ndarray, rank: int):
    """Method of snapshots on X (N x m, columns are snapshots).

    Returns (mean, basis N x rank, singular values of the centred snapshots).
    """
    mean = X.mean(axis=1)
    Xc = X - mean[:, None]
    C = Xc.T @ Xc
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1]
    lam = np.clip(lam[order], 0.0, None)
    V = V[:, order]
    r = min(rank, int(np.sum(lam > lam[0] * 1e-28)) if lam[0] > 0 else 0)
    B = Xc @ V[:, :r] / np.sqrt(lam[:r])[None, :]
    if r < rank:
        B = np.concatenate([B, np.zeros((X.shape[0], rank - r))], axis=1)
    return mean, B, np.sqrt(lam)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def mlp_init(sizes=(3, 256, 256, 64), seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = rng.normal(0.0, math.sqrt(2.0 / a), size=(b, a))
        params.append([W, np.zeros(b)])
    return params


def mlp_forward(params, x):
    """x: B x 3.  Returns output and the cache for backward."""
    cache = []
    h = x
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        cache.append((h, z))
        h = gelu(z) if li < len(params) - 1 else z
    return h, cache


def bf16_round(x):
    """Round FP32 values to bfloat16 (keep the top 16 bits of the FP32 pattern, ties to
    even), returned as float64.  Inputs are first rounded to FP32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_forward_bf16(params, x):
    """mlp_forward with the weights and each layer's input rounded to bfloat16; products
    summed exactly (FP64), biases kept FP32."""
    h = np.asarray(x, dtype=float)
    for li, (W, b) in enumerate(params):
        z = bf16_round(h) @ bf16_round(W).T + np.asarray(b, dtype=np.float32).astype(float)
        h = gelu(z) if li < len(params) - 1 else z
    return h


def mlp_loss(params, x, t):
    y, _ = mlp_forward(params, x)
    return float(np.mean((y - t) ** 2))


def mlp_backward(params, x, t):
    """Gradients of the mean squared error (mean over batch and outputs)."""
    y, cache = mlp_forward(params, x)
    g = 2.0 * (y - t) / y.size
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        h_in, z = cache[li]
        if li < len(params) - 1:
            g = g * gelu_grad(z)
        W, _b = params[li]
        grads[li] = [g.T @ h_in, g.sum(axis=0)]
        g = g @ W
    return grads


def adamw_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=1e-4):
    """Decoupled-weight-decay Adam; state = {'t': int, 'm': [...], 'v': [...]}."""
    if not state:
        state.update(t=0, m=[[np.zeros_like(p) for p in lp] for lp in params],
                     v=[[np.zeros_like(p) for p in lp] for lp in params])
    state["t"] += 1
    t = state["t"]
    for li, lp in enumerate(params):
        for pi, p in enumerate(lp):
            g = grads[li][pi]
            m = state["m"][li][pi] = b1 * state["m"][li][pi] + (1 - b1) * g
            v = state["v"][li][pi] = b2 * state["v"][li][pi] + (1 - b2) * g * g
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            lp[pi] = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return params

"""Comparison helpers of the GPU parity tests."""
import numpy as np


def rel(a, b):
    """Normwise relative difference ||a - b|| / ||b||."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elementwise(a, b, tol, n=None):
    """Largest |a - b| / (|b| + scale of b's row block): every entry is held to tol relative to
    itself or to the largest entry of its block, so small entries cannot hide behind a norm.
    With n given, a state array [2n][...] has the two row blocks q and u; a sensitivity matrix
    [2n][2n] has the four blocks dq/dq0, dq/du0, du/dq0, du/du0."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    scale = np.zeros_like(b)
    if n is None:
        scale[...] = np.abs(b).max()
    elif b.ndim >= 2 and b.shape[-1] == 2 * n and b.shape[-2] == 2 * n:
        for r in (slice(0, n), slice(n, 2 * n)):
            for c in (slice(0, n), slice(n, 2 * n)):
                scale[..., r, c] = np.abs(b[..., r, c]).max()
    else:
        for r in (slice(0, n), slice(n, 2 * n)):
            scale[r] = np.abs(b[r]).max()
    err = np.abs(a - b) / (np.abs(b) + scale + 1e-300)
    worst = float(err.max())
    assert worst <= tol, f"elementwise error {worst:.3e} > {tol:.1e} at {np.unravel_index(err.argmax(), err.shape)}"
    return worst

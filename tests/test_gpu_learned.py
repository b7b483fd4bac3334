"""GPU learned predictor: snapshot POD, MLP loss/gradients and AdamW against the oracle,
and what the trained predictor gains over the secant predictor in a continuation sweep."""
import numpy as np
import pytest

from fse_inputs import Torus, tiny_system
from oracle import learned as olearn
from oracle import shooting as osh

pytestmark = pytest.mark.gpu
GOLDEN = (1 + 5 ** 0.5) / 2


def fse():
    import paper_2508_06302_amd as m
    return m


def log(msg):
    print(msg, flush=True)


def _ctx(K=40, S=96):
    s = tiny_system(n=3, seed=2, cubic=1.0, quad=0.3, e=2)
    tr = Torus(d=2, e=2, K=[np.arange(1, K)], S=[S], S1=64)
    return s, tr, fse().fse_init_torus(s, tr)


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def _unflat(flat, sizes):
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = flat[o:o + a * b].reshape(b, a)
        o += a * b
        bias = flat[o:o + b]
        o += b
        out.append([W.astype(np.float64), bias.astype(np.float64)])
    return out


def test_pod_matches_oracle_snapshots():
    """Singular values, mean and the spanned subspace of the leading modes (modes are
    defined up to sign) against the oracle's method of snapshots."""
    s, tr, ctx = _ctx()
    N = 2 * ctx.n * ctx.U
    rng = np.random.default_rng(3)
    m, rank = 30, 12
    basis = np.linalg.qr(rng.normal(size=(N, 15)))[0]
    X = (basis * (0.5 ** np.arange(15))) @ rng.normal(size=(15, m)) + 1e-3 * rng.normal(size=(N, 1))
    mean_o, B_o, sig_o = olearn.pod_snapshots(X, rank)
    lp = fse().fse_learned_create(ctx, n_in=3, hidden=16, rank=rank)
    sig = lp.fit_pod(X.T.copy())
    mean, modes = lp.get_pod()
    mean, modes = mean.cpu().numpy(), modes.cpu().numpy()
    assert np.abs(sig - sig_o[:rank]).max() < 1e-10 * sig_o[0]
    assert np.abs(mean - mean_o).max() < 1e-14 * np.abs(X).max()
    # leading modes with separated singular values: same column up to sign
    for r in range(8):
        c = abs(float(modes[:, r] @ B_o[:, r]))
        assert abs(c - 1.0) < 1e-9, (r, c)
    assert np.abs(modes.T @ modes - np.eye(rank)).max() < 1e-10


@pytest.mark.parametrize("sizes", [(3, 16, 16, 4), (3, 256, 256, 64)])
def test_mlp_loss_and_gradients_match_oracle(sizes):
    """Hand-written FP32 forward/backward vs the oracle's FP64 backward at the same
    (FP32-representable) weights."""
    s, tr, ctx = _ctx(K=6, S=16)
    lp = fse().fse_learned_create(ctx, n_in=sizes[0], hidden=sizes[1], rank=sizes[3])
    params = olearn.mlp_init(sizes, seed=5)
    flat = _flat(params).astype(np.float32)
    lp.set_params(flat)
    p32 = _unflat(flat, sizes)
    rng = np.random.default_rng(9)
    x = rng.normal(size=(24, sizes[0])).astype(np.float32)
    t = rng.normal(size=(24, sizes[3])).astype(np.float32)
    loss, g = lp.loss_grad(x, t)
    lo = olearn.mlp_loss(p32, x.astype(np.float64), t.astype(np.float64))
    go = _flat(olearn.mlp_backward(p32, x.astype(np.float64), t.astype(np.float64)))
    log(f"sizes {sizes}: loss {loss:.6e} vs {lo:.6e}; grad rel err "
        f"{np.linalg.norm(g - go) / np.linalg.norm(go):.2e}")
    assert abs(loss - lo) < 1e-5 * lo
    assert np.linalg.norm(g - go) < 1e-4 * np.linalg.norm(go)


def test_adamw_steps_match_oracle():
    """Twenty full-batch AdamW steps on the GPU (FP32) and in the oracle (FP64) from the
    same start: same loss history and parameters to FP32 accuracy."""
    sizes = (3, 32, 32, 8)
    s, tr, ctx = _ctx(K=6, S=16)
    lp = fse().fse_learned_create(ctx, n_in=3, hidden=32, rank=8)
    params = olearn.mlp_init(sizes, seed=6)
    flat = _flat(params).astype(np.float32)
    lp.set_params(flat)
    rng = np.random.default_rng(10)
    x = rng.normal(size=(40, 3)).astype(np.float32)
    t = np.tanh(x @ rng.normal(size=(3, 8))).astype(np.float32)
    hist = lp.fit(x, t, steps=20, lr=1e-3, wd=1e-4)
    po = _unflat(flat, sizes)
    state, ho = {}, []
    for _ in range(20):
        ho.append(olearn.mlp_loss(po, x.astype(np.float64), t.astype(np.float64)))
        g = olearn.mlp_backward(po, x.astype(np.float64), t.astype(np.float64))
        po = olearn.adamw_step(po, g, state, lr=1e-3, wd=1e-4)
    assert np.abs(hist - np.array(ho)).max() < 1e-4 * max(ho)
    # Adam normalises every component, so a gradient component within FP32 rounding of zero
    # may step either way: compare the parameter updates as a whole
    got = lp.get_params().astype(np.float64)
    ref = _flat(po)
    du_g, du_o = got - flat, ref - flat
    err = np.linalg.norm(du_g - du_o) / np.linalg.norm(du_o)
    log(f"AdamW: loss {ho[0]:.4e} -> {hist[-1]:.4e}; update rel diff vs FP64 oracle {err:.2e}")
    assert err < 1e-2


def _grid(w_lo, w_hi, f_lo, f_hi, nw, nf, offset=0.0):
    dw, df = (w_hi - w_lo) / (nw - 1), (f_hi - f_lo) / (nf - 1)
    pts = []
    for i in range(nf):
        f = f_lo + (i + offset) * df
        ws = [w_lo + (k + offset) * dw for k in range(nw)]
        pts += [(w, f) for w in (ws if i % 2 == 0 else ws[::-1])]
    return pts


def test_learned_predictor_gains_over_secant():
    """Continuation sweep on the 3-DOF system (d = 2, forcing ratio the golden mean):
    100 points on a serpentine in (omega_1, f) train the POD + MLP predictor; 100 points
    interleaved with them are then solved (a) in serpentine order and (b) in a seeded
    random order, once with the secant predictor alone and once with the learned
    predictor judged against it.  Gains are Newton iterations to ||R|| < 1e-10."""
    m = fse()
    s = tiny_system(n=3, seed=2, cubic=1.0, quad=0.3, e=2)
    tr = Torus(d=2, e=2, K=[np.arange(1, 6)], S=[16], S1=64)
    ctx = m.fse_init_torus(s, tr)
    train = _grid(0.40, 0.55, 0.10, 0.40, 10, 10)
    evalp = _grid(0.40, 0.55, 0.10, 0.40, 10, 10, offset=0.5)
    evalp = [(w, f) for (w, f) in evalp if w <= 0.55 and f <= 0.40]

    def params(pts):
        return np.array([[w, GOLDEN * w, f, f] for (w, f) in pts])

    def feats(pts):
        return np.array([[w, GOLDEN, f] for (w, f) in pts])

    Z0 = np.zeros((6, ctx.U))
    Zt, it_t, rn_t = m.fse_continuation(ctx, params(train), Z0, tol=1e-10, maxit=20)
    assert np.all(rn_t < 1e-10)
    lp = m.fse_learned_create(ctx, n_in=3, hidden=256, rank=64)
    params_mlp = olearn.mlp_init((3, 256, 256, 64), seed=7)
    lp.set_params(_flat(params_mlp).astype(np.float32))
    lp.fit_pod(Zt)
    hist = lp.train(feats(train), Zt, epochs=3000, lr=1e-3, wd=1e-5)
    log(f"training loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < 1e-2 * hist[0]
    rng = np.random.default_rng(12)
    results = {}
    for order in ("serpentine", "shuffled"):
        pts = list(evalp) if order == "serpentine" else [evalp[i] for i in rng.permutation(len(evalp))]
        _, it_s, rn_s = m.fse_continuation(ctx, params(pts), Zt[-1], tol=1e-10, maxit=20)
        _, it_l, rn_l, used = m.fse_continuation_learned(ctx, params(pts), feats(pts), Zt[-1], lp, 0,
                                                         tol=1e-10, maxit=20)
        assert np.all(rn_s < 1e-10) and np.all(rn_l < 1e-10)
        results[order] = (it_s.mean(), it_l.mean(), used.mean())
        log(f"{order}: Newton iterations per point secant {it_s.mean():.2f}, "
            f"learned+judge {it_l.mean():.2f} (learned prediction taken at {100 * used.mean():.0f}% "
            f"of the points)")
    assert results["shuffled"][1] < results["shuffled"][0]
    assert results["serpentine"][1] <= results["serpentine"][0] + 0.05


@pytest.mark.parametrize("sizes,B", [((3, 256, 256, 64), 100), ((3, 40, 40, 10), 7)])
def test_bf16_mfma_forward_matches_the_bf16_oracle(sizes, B):
    """BF16 matrix-core inference: equal to the oracle's forward with bfloat16-rounded
    weights and layer inputs up to FP32 accumulation (which can move a layer input to the
    neighbouring bfloat16), and within bfloat16 accuracy of the FP32 network (ragged tiles:
    B and the widths are not multiples of 16)."""
    s, tr, ctx = _ctx(K=6, S=16)
    lp = fse().fse_learned_create(ctx, n_in=sizes[0], hidden=sizes[1], rank=sizes[3])
    params = olearn.mlp_init(sizes, seed=11)
    flat = _flat(params).astype(np.float32)
    lp.set_params(flat)
    p32 = _unflat(flat, sizes)
    x = np.random.default_rng(13).normal(size=(B, sizes[0])).astype(np.float32)
    yb = lp.forward(x, bf16=True).astype(np.float64)
    yf = lp.forward(x, bf16=False).astype(np.float64)
    ob = olearn.mlp_forward_bf16(p32, x.astype(np.float64))
    of, _ = olearn.mlp_forward(p32, x.astype(np.float64))
    eb = np.linalg.norm(yb - ob) / np.linalg.norm(ob)
    ef = np.linalg.norm(yb - of) / np.linalg.norm(of)
    log(f"sizes {sizes} B={B}: bf16 MFMA vs bf16 oracle {eb:.2e}, vs FP32 network {ef:.2e}, "
        f"FP32 path vs oracle {np.linalg.norm(yf - of) / np.linalg.norm(of):.2e}")
    # FP32 sums may round a layer input to the neighbouring bfloat16 now and then
    assert eb < 1e-3
    assert ef < 3e-2


def test_batch_prediction_matches_single_predictions():
    """predict_batch (FP32) equals predict point by point; the BF16 batch agrees to
    bfloat16 accuracy on the POD coefficients."""
    s, tr, ctx = _ctx(K=6, S=16)
    N = 2 * ctx.n * ctx.U
    rng = np.random.default_rng(21)
    P = np.column_stack([np.linspace(0.4, 0.6, 24), np.full(24, GOLDEN), np.linspace(0.1, 0.3, 24)])
    X = np.array([np.sin(3 * p[0]) * np.cos(np.arange(N) * p[2]) + p[2] * np.arange(N) / N for p in P])
    lp = fse().fse_learned_create(ctx, n_in=3, hidden=32, rank=8)
    lp.set_params(_flat(olearn.mlp_init((3, 32, 32, 8), seed=3)).astype(np.float32))
    lp.fit_pod(X)
    lp.train(P, X, epochs=200, lr=1e-3, wd=1e-5)
    Q = P[::5] + 0.003
    Zb = lp.predict_batch(Q).cpu().numpy()
    Zs = np.stack([lp.predict(q).cpu().numpy() for q in Q])
    assert np.abs(Zb - Zs).max() <= 1e-12 * np.abs(Zs).max()
    Zh = lp.predict_batch(Q, bf16=True).cpu().numpy()
    mean, modes = lp.get_pod()
    mean, modes = mean.cpu().numpy(), modes.cpu().numpy()
    cb = (Zh.reshape(len(Q), -1) - mean) @ modes
    cs = (Zs.reshape(len(Q), -1) - mean) @ modes
    err = np.linalg.norm(cb - cs) / np.linalg.norm(cs)
    log(f"BF16 batch vs FP32 predictions: POD coefficients rel diff {err:.2e}")
    assert err < 3e-2

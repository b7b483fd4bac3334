"""Pins of the oracle's torus bookkeeping (App. B, App. D, Eqs. 13-14, 19, 24)."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import torus as tor

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_counts():
    rows = []
    with open(os.path.join(GOLD, "unknown_counts.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            sec, n, klists, count, kind = line.split()
            ks = [np.array([int(v) for v in part.split(",")]) for part in klists.split(";")]
            rows.append((sec, int(n), ks, int(count), kind))
    return rows


@pytest.mark.parametrize("row", _read_counts(), ids=lambda r: f"{r[0]}-{r[3]}")
def test_printed_unknown_counts(row):
    """Sec. 4: printed numbers of unknowns pin U~ = prod(2 L_j + 1) and the table size."""
    sec, n, ks, count, kind = row
    if kind == "fse":
        U = tor.n_coefficients(ks)
        assert 2 * n * U == count
        T = tor.harmonic_table(ks)
        assert T.shape == ((U + 1) // 2, len(ks))
        assert not T[-1].any()
    else:
        assert n * tor.n_coefficients(ks) == count


def _box(klists):
    axes = [sorted(set([0] + list(k) + [-v for v in k])) for k in klists]
    return set(itertools.product(*axes))


@pytest.mark.parametrize("klists", [
    [[1, 3]], [[1, 2, 3, 4, 5]],
    [[1, 3], [1, 3]], [[1, 2], [1, 2, 3]], [[1, 3], [1, 3], [1, 3]],
    [list(range(1, 9)), list(range(1, 9))],
])
def test_table_tiles_box_once(klists):
    """App. B: every harmonic of the box appears exactly once as +row or -row (brute force)."""
    T = tor.harmonic_table([np.array(k) for k in klists])
    rows = [tuple(int(v) for v in r) for r in T[:-1]]
    seen = []
    for r in rows:
        seen.append(r)
        seen.append(tuple(-v for v in r))
    assert len(seen) == len(set(seen))
    assert set(seen) | {tuple([0] * len(klists))} == _box(klists)
    assert tuple(int(v) for v in T[-1]) == tuple([0] * len(klists))
    assert (0,) * len(klists) not in rows


def test_table_blocks_d3():
    """App. B for d = 3 (K_2 = K_3 = [0..8]): 64 g-rows (k_2 > 0, k_3 < 0) then 81 b-rows (k_3 >= 0)."""
    k = np.arange(1, 9)
    T = tor.harmonic_table([k, k])
    assert T.shape == (145, 2)
    g, b = T[:64], T[64:]
    assert (g[:, 0] > 0).all() and (g[:, 1] < 0).all()
    assert (b[:, 1] >= 0).all()
    # b-block: outer loop over [k_3; 0], inner over K~^2 = [k_2; 0]
    assert tuple(b[0]) == (1, 1) and tuple(b[8]) == (0, 1) and tuple(b[-1]) == (0, 0)


def test_sample_order_phi2_fastest():
    """Eq. (D1): phi_2 varies fastest, then phi_3."""
    idx = tor.sample_indices([3, 2])
    assert idx[0].tolist() == [0, 1, 2, 0, 1, 2]
    assert idx[1].tolist() == [0, 0, 0, 1, 1, 1]


@pytest.mark.parametrize("klists,S", [([range(1, 6)], [16]), ([range(1, 6)], [11]),
                                      ([range(1, 4), range(1, 3)], [8, 5]),
                                      ([[1, 3], [1, 3], [2]], [7, 7, 5])])
def test_gamma_inverse_identity(klists, S):
    """Gamma^-1 Gamma = I when S_j >= 2 H_j + 1 (Nyquist condition of Sec. 3.1)."""
    T = tor.harmonic_table([np.array(list(k)) for k in klists])
    G, Gi = tor.gamma_matrices(T, S)
    assert np.allclose(Gi @ G, np.eye(G.shape[1]), atol=1e-13)


def test_gamma_aliasing_below_nyquist():
    T = tor.harmonic_table([np.arange(1, 6)])
    G, Gi = tor.gamma_matrices(T, [9])
    assert not np.allclose(Gi @ G, np.eye(11), atol=1e-6)


def test_gamma_inverse_vs_numpy_fft_d2():
    """Gamma^-1 = real DFT: constant = F_0/S, cos = 2 Re F_k / S, sin = -2 Im F_k / S."""
    rng = np.random.default_rng(3)
    S = 32
    T = tor.harmonic_table([np.arange(1, 11)])
    _, Gi = tor.gamma_matrices(T, [S])
    x = rng.normal(size=S)
    F = np.fft.fft(x)
    c = Gi @ x
    assert np.isclose(c[0], F[0].real / S, atol=1e-14)
    for l, k in enumerate(T[:-1, 0]):
        assert np.isclose(c[2 * l + 1], 2 * F[k].real / S, atol=1e-14)
        assert np.isclose(c[2 * l + 2], -2 * F[k].imag / S, atol=1e-14)


def test_gamma_inverse_vs_numpy_fftn_d3():
    rng = np.random.default_rng(4)
    S2, S3 = 8, 6
    T = tor.harmonic_table([np.arange(1, 4), np.arange(1, 3)])
    _, Gi = tor.gamma_matrices(T, [S2, S3])
    x = rng.normal(size=S2 * S3)
    F = np.fft.fftn(x.reshape(S3, S2))          # phi_2 fastest -> last axis
    c = Gi @ x
    St = S2 * S3
    assert np.isclose(c[0], F[0, 0].real / St, atol=1e-14)
    for l, (k2, k3) in enumerate(T[:-1]):
        f = F[k3 % S3, k2 % S2]
        assert np.isclose(c[2 * l + 1], 2 * f.real / St, atol=1e-14)
        assert np.isclose(c[2 * l + 2], -2 * f.imag / St, atol=1e-14)


def test_gamma_rows_are_trig_basis():
    """Row s of Gamma is H(k~, phi~_s) of Eq. (11)."""
    T = tor.harmonic_table([np.arange(1, 4), np.arange(1, 3)])
    G, _ = tor.gamma_matrices(T, [8, 5])
    ang = tor.sample_angles([8, 5])
    for s in (0, 7, 13, 39):
        assert np.allclose(G[s], tor.trig_row(T, ang[:, s]), atol=1e-14)


@pytest.mark.parametrize("klists", [[range(1, 6)], [range(1, 4), range(1, 3)],
                                    [[1, 3], [1, 3], [1, 3]]])
def test_rotation_is_phase_shift(klists):
    """Eq. (13): H(phi~ - 2 pi rho) = H(phi~) R(rho), pointwise."""
    rng = np.random.default_rng(5)
    T = tor.harmonic_table([np.array(list(k)) for k in klists])
    d1 = T.shape[1]
    for _ in range(5):
        phi = rng.uniform(0, 2 * np.pi, d1)
        rho = rng.uniform(-2, 2, d1)
        R = tor.rotation(T, rho)
        lhs = tor.trig_row(T, phi - 2 * np.pi * rho)
        assert np.allclose(lhs, tor.trig_row(T, phi) @ R, atol=1e-12)
        assert np.allclose(R.T @ R, np.eye(R.shape[0]), atol=1e-13)
        assert np.allclose(tor.rotation(T, rho + 1.0), R, atol=1e-11)


def test_nabla_is_phase_derivative():
    """Eq. (19): d/dphi_i [H(phi~) Z] = H(phi~) (nabla_i Z)."""
    rng = np.random.default_rng(6)
    T = tor.harmonic_table([np.arange(1, 4), np.arange(1, 3)])
    Z = rng.normal(size=T.shape[0] * 2 - 1)
    phi = rng.uniform(0, 2 * np.pi, 2)
    h = 1e-6
    for i in (2, 3):
        e = np.zeros(2)
        e[i - 2] = h
        fd = (tor.trig_row(T, phi + e) @ Z - tor.trig_row(T, phi - e) @ Z) / (2 * h)
        assert np.isclose(fd, tor.trig_row(T, phi) @ (tor.nabla(T, i) @ Z), rtol=1e-8, atol=1e-8)


@pytest.mark.parametrize("d", [2, 3])
def test_rotation_domega_matches_fd(d):
    """Eq. (24) with the 2 pi / omega_1 reading, against central differences in omega_i."""
    T = tor.harmonic_table([np.arange(1, 4)] * (d - 1))
    om = np.array([1.3, 2.1, 0.7][:d])
    h = 1e-6
    for i in range(1, d + 1):
        e = np.zeros(d)
        e[i - 1] = h
        fd = (tor.rotation(T, (om + e)[1:] / (om + e)[0])
              - tor.rotation(T, (om - e)[1:] / (om - e)[0])) / (2 * h)
        assert np.allclose(tor.rotation_domega(T, om, i), fd, atol=1e-7)

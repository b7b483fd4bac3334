"""Torus discretisation of FSE-Shooting (oracle; test infrastructure only).

Pins (tests/test_oracle_torus.py): printed unknown counts of Secs. 4.1-4.3,
tiling of the harmonic box by +/- rows (brute force), Gamma^-1 Gamma = I,
Gamma^-1 against numpy.fft / fftn, the shift identity that defines R(rho)
(Eq. 13), finite differences of R(rho) in omega.
"""
from __future__ import annotations

import math

import numpy as np


def harmonic_table(k_lists) -> np.ndarray:
    """Matrix K~^d of App. B (Eqs. B1-B2).

    k_lists[j-2] holds the positive harmonic orders k_j of direction j
    (K_j = [0; k_j]).  For d = 2 the table is [k_2; 0].  For d > 2 it is built
    from K~^{d-1} = [K~^{d-1,r}; 0]:
      g-block: for every -k in -k_d, every row r of K~^{d-1,r}:   [r, -k]
      b-block: for every k in [k_d; 0], every row r of K~^{d-1}:  [r,  k]
    (e_m (x) X stacks m copies of X; v (x) e_m repeats every entry of v m times.)
    Rows 0..L-1 are the harmonic vectors k~_1..k~_L; the last row is zero.
    """
    if len(k_lists) == 0:
        return np.zeros((1, 0), dtype=np.int64)
    k2 = np.asarray(k_lists[0], dtype=np.int64)
    T = np.concatenate([k2[:, None], np.zeros((1, 1), np.int64)], axis=0)
    for kd in k_lists[1:]:
        kd = np.asarray(kd, dtype=np.int64)
        Ld = len(kd)
        Tr = T[:-1]
        Lp = len(Tr)
        g = np.concatenate([np.tile(Tr, (Ld, 1)), np.repeat(-kd, Lp)[:, None]], axis=1)
        kd0 = np.concatenate([kd, [0]])
        b = np.concatenate([np.tile(T, (Ld + 1, 1)), np.repeat(kd0, Lp + 1)[:, None]], axis=1)
        T = np.concatenate([g, b], axis=0)
    return T


def n_coefficients(k_lists) -> int:
    """U~ = prod_j (2 L_j + 1)  (Sec. 3.1)."""
    u = 1
    for k in k_lists:
        u *= 2 * len(k) + 1
    return u


def sample_indices(S_list) -> np.ndarray:
    """Integer sample coordinates s_j of every grid point, shape (d-1, S~) (Eq. D1).

    T_j = e^T_{S_{j+1}..S_d} (x) phibar_j (x) e^T_{S_2..S_{j-1}}: phi_2 varies fastest.
    """
    S = [int(v) for v in S_list]
    total = int(np.prod(S)) if S else 1
    idx = np.zeros((len(S), total), dtype=np.int64)
    for j in range(len(S)):
        inner = int(np.prod(S[:j])) if j > 0 else 1
        outer = int(np.prod(S[j + 1:])) if j + 1 < len(S) else 1
        idx[j] = np.tile(np.repeat(np.arange(S[j]), inner), outer)
    return idx


def sample_angles(S_list) -> np.ndarray:
    """phi~_s = 2 pi s_j / S_j, shape (d-1, S~)."""
    idx = sample_indices(S_list)
    S = np.asarray(S_list, dtype=float).reshape(-1, 1)
    return 2.0 * np.pi * idx / S


def harmonic_angles(table: np.ndarray, S_list) -> np.ndarray:
    """k~_l . phi~_s for l = 1..L, shape (S~, L), reduced exactly in integers.

    The sum of fractions sum_j (k_{j,l} s_j mod S_j) / S_j is formed over the
    common denominator prod S_j before a single division.
    """
    idx = sample_indices(S_list)
    S = [int(v) for v in S_list]
    P = int(np.prod(S))
    L = table.shape[0] - 1
    num = np.zeros((idx.shape[1], L), dtype=np.int64)
    for j in range(len(S)):
        kj = table[:L, j].astype(np.int64)
        part = np.mod(np.outer(idx[j], kj), S[j]) * (P // S[j])
        num = np.mod(num + part, P)
    return 2.0 * np.pi * num.astype(float) / P


def gamma_matrices(table: np.ndarray, S_list):
    """Gamma (S~ x U~, Eq. D2) and Gamma^-1 (U~ x S~, Eq. D3).

    Column order [1, cos k~_1.phi~, sin k~_1.phi~, ..., cos k~_L.phi~, sin k~_L.phi~].
    """
    th = harmonic_angles(table, S_list)
    Stil, L = th.shape
    U = 2 * L + 1
    G = np.empty((Stil, U))
    G[:, 0] = 1.0
    G[:, 1::2] = np.cos(th)
    G[:, 2::2] = np.sin(th)
    Gi = np.empty((U, Stil))
    Gi[0, :] = 1.0 / Stil
    Gi[1::2, :] = 2.0 * np.cos(th).T / Stil
    Gi[2::2, :] = 2.0 * np.sin(th).T / Stil
    return G, Gi


def trig_row(table: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """H(k~, phi~) of Eq. (11) at one point phi~ (length d-1)."""
    L = table.shape[0] - 1
    th = table[:L].astype(float) @ np.asarray(phi, dtype=float)
    h = np.empty(2 * L + 1)
    h[0] = 1.0
    h[1::2] = np.cos(th)
    h[2::2] = np.sin(th)
    return h


def rotation(table: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """R(rho) of Eq. (14): 2x2 rotation by alpha_l = 2 pi k~_l . rho per harmonic pair."""
    L = table.shape[0] - 1
    U = 2 * L + 1
    R = np.zeros((U, U))
    R[0, 0] = 1.0
    alpha = 2.0 * np.pi * (table[:L].astype(float) @ np.asarray(rho, dtype=float))
    for l in range(L):
        c, s = math.cos(alpha[l]), math.sin(alpha[l])
        a, b = 2 * l + 1, 2 * l + 2
        R[a, a], R[a, b] = c, -s
        R[b, a], R[b, b] = s, c
    return R


def nabla(table: np.ndarray, i: int) -> np.ndarray:
    """nabla_{phi_i} of Eq. (19), i = 2..d: blocks [[0, k_{i,l}], [-k_{i,l}, 0]]."""
    L = table.shape[0] - 1
    U = 2 * L + 1
    N = np.zeros((U, U))
    for l in range(L):
        k = float(table[l, i - 2])
        a, b = 2 * l + 1, 2 * l + 2
        N[a, b] = k
        N[b, a] = -k
    return N


def rotation_domega(table: np.ndarray, omega: np.ndarray, i: int) -> np.ndarray:
    """dR(rho)/d omega_i of Eq. (24), i = 1..d (1-based), with rho_j = omega_j / omega_1.

    Reading of Eq. (24): the prefactor is 2 pi / omega_1 for every i, which is
    d alpha_l / d omega_i for alpha_l = 2 pi sum_j k_{j,l} omega_j / omega_1 (the
    printed 2 pi / omega_i is read as a typo for i >= 2; the i = 1 line agrees).
    """
    omega = np.asarray(omega, dtype=float)
    rho = omega[1:] / omega[0]
    L = table.shape[0] - 1
    U = 2 * L + 1
    Ups = np.zeros((U, U))
    for l in range(L):
        if i == 1:
            kr = float(table[l].astype(float) @ rho)
            blk = -np.array([[0.0, -kr], [kr, 0.0]])
        else:
            k = float(table[l, i - 2])
            blk = np.array([[0.0, -k], [k, 0.0]])
        a = 2 * l + 1
        Ups[a:a + 2, a:a + 2] = blk
    return (2.0 * np.pi / omega[0]) * Ups @ rotation(table, rho)

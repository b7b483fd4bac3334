"""Matrix-free Newton-Krylov step of the shooting problem (oracle; test infrastructure only).

For unknown counts where the dense Jacobian of Eq. (22) is too large to factor, the Newton
correction is found with GMRES.  The Jacobian is then only applied to vectors, in the order
in which Eq. (22) composes it:
    J v = (I (x) R(rho) Gamma^-1) blkdiag_s(Phi_s) (I (x) Gamma) v - v.

Preconditioner (harmonic blocks): P = Phi_bar (x) R(rho) - I, where Phi_bar is the mean of
the trajectory sensitivities Phi_s.  Each Phi_s of a linear system is the same matrix, and
Gamma^-1 Gamma = I.  So for a linear system P equals J exactly (the closed form J = Phi (x)
R - I of the linear case).  R(rho) is block-diagonal: a 1 x 1 block for the zero harmonic
and a 2 x 2 rotation per harmonic pair.  So P splits into one 2n x 2n block and one
4n x 4n block per pair, and P^-1 is a set of small dense solves.

GMRES: restarted GMRES(m) with right preconditioning, modified Gram-Schmidt Arnoldi and
Givens rotations on the Hessenberg matrix (Saad and Schultz, 1986).  The stop is the
true residual ||J x + R|| <= rtol ||R||, checked at every restart.

Pins (tests/test_oracle_krylov.py): J v against the dense Jacobian; on a linear system the
preconditioned operator is the identity and GMRES converges in one iteration; on nonlinear
systems the correction meets its tolerance against a dense solve, and Newton-Krylov reaches
the torus of dense Newton.
"""
from __future__ import annotations

import numpy as np

from . import shooting


def jacobian_apply(res, v):
    """J v for v of shape [2n][U~] (Eq. 22 applied to a vector)."""
    tb = res["tables"]
    Phi = res["Phi"]                       # [S~][2n][2n]
    x = np.asarray(v, dtype=float) @ tb.G.T          # [2n][S~] = (I (x) Gamma) v
    y = np.einsum("sij,js->is", Phi, x)               # blkdiag(Phi_s) x
    return (y @ tb.Gi.T) @ res["Rrot"].T - v          # (I (x) R Gamma^-1) y - v


def harmonic_blocks(res):
    """Blocks of P = Phi_bar (x) R(rho) - I: list of (unknown indices, dense block)."""
    Phib = res["Phi"].mean(axis=0)
    Rm = res["Rrot"]
    U = Rm.shape[0]
    n2 = Phib.shape[0]
    groups = [[0]] + [[2 * l + 1, 2 * l + 2] for l in range((U - 1) // 2)]
    blocks = []
    for g in groups:
        idx = [i * U + a for i in range(n2) for a in g]
        B = np.kron(Phib, Rm[np.ix_(g, g)]) - np.eye(len(idx))
        blocks.append((np.array(idx), B))
    return blocks


def precondition(blocks, r):
    """P^-1 r for r of shape [2n][U~]."""
    shape = np.shape(r)
    flat = np.ravel(r)
    out = np.empty_like(flat)
    for idx, B in blocks:
        out[idx] = np.linalg.solve(B, flat[idx])
    return out.reshape(shape)


def gmres(apply_A, b, rtol=1e-10, restart=30, maxit=300, apply_M=None):
    """Solve A x = b, x0 = 0, right-preconditioned by M^-1 (apply_M) if given.
    Returns (x, iterations, ||b - A x|| / ||b||)."""
    b = np.asarray(b, dtype=float)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, 0.0
    M = apply_M if apply_M is not None else (lambda v: v)
    its = 0
    while True:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * nb or its >= maxit:
            return x, its, beta / nb
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k = 0
        for k in range(restart):
            w = apply_A(M(V[k]))
            for j in range(k + 1):
                H[j, k] = np.vdot(V[j], w)
                w = w - H[j, k] * V[j]
            H[k + 1, k] = np.linalg.norm(w)
            V.append(w / H[k + 1, k] if H[k + 1, k] > 0 else w)
            for j in range(k):
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
                H[j, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            its += 1
            if abs(g[k + 1]) <= rtol * nb or its >= maxit:
                break
        m = k + 1
        y = np.linalg.solve(np.triu(H[:m, :m]), g[:m])
        x = x + M(sum(yj * vj for yj, vj in zip(y, V[:m])))


def newton_krylov_step(sysm, torus, omega, Z0, rtol=1e-10, restart=30, maxit=300, precond=True,
                       tables=None, tol=1e-12):
    """One Newton update Z0 -> Z0 + dZ with J dZ = -R solved by GMRES (d = e).
    Returns (Z_new, ||R||_2 before the update, GMRES iterations, relative residual)."""
    tb = tables or shooting.TorusTables(torus)
    res = shooting.evaluate(sysm, torus, omega, Z0, sens=True, tables=tb, tol=tol)
    R = res["R"]
    blocks = harmonic_blocks(res) if precond else None
    dZ, its, rel = gmres(lambda v: jacobian_apply(res, v), -R, rtol=rtol, restart=restart, maxit=maxit,
                         apply_M=(lambda v: precondition(blocks, v)) if precond else None)
    return Z0 + dZ, float(np.linalg.norm(R)), its, rel

"""Seeded systems with velocity-dependent forces (factor index n + j names qdot_j)."""
import numpy as np

from fse_inputs import tiny_system
from fse_inputs.systems import System


def van_der_pol(mu=0.2, F=0.5):
    """q'' - mu (1 - q^2) q' + q = F cos(omega_1 t): D = -mu, f_nl = mu q^2 qdot."""
    return System("van_der_pol", np.eye(1), np.array([[-mu]]), np.eye(1), np.zeros((0, 3), np.int32),
                  np.zeros(0), np.array([[0, 0, 0, 1]], np.int32), np.array([mu]), np.array([[F]]))


def mixed_system(n=3, seed=2, e=2, eps=0.4, mu=0.3):
    """tiny_system plus f_i += mu_i q_i^2 qdot_i + eps g_i (g.q)^2 (g.qdot): both tangents
    d f / d q and d f / d qdot are symmetric."""
    s = tiny_system(n=n, seed=seed, cubic=1.0, quad=0.3, e=e)
    g = np.random.default_rng(seed + 100).normal(size=n) / np.sqrt(n)
    idx, val = [list(r) for r in s.t3_idx], list(s.t3_val)
    for i in range(n):
        idx.append([i, i, i, n + i])
        val.append(mu * (1.0 + 0.5 * i))
        for j in range(n):
            for k in range(n):
                for l in range(n):
                    idx.append([i, j, k, n + l])
                    val.append(eps * g[i] * g[j] * g[k] * g[l])
    s.t3_idx = np.array(idx, np.int32)
    s.t3_val = np.array(val)
    return s


def with_contacts(s, dof, direction, gap, k):
    """Copy of s with unilateral penalty contacts (dof, direction +-1, gap, stiffness)."""
    import dataclasses
    return dataclasses.replace(s, con_dof=np.asarray(dof, np.int32), con_dir=np.asarray(direction, np.int32),
                               con_gap=np.asarray(gap, float), con_k=np.asarray(k, float))


def impact_oscillator(c=0.2, kc=4.0, gap=0.3, F=0.6, two_sided=False):
    """q'' + c q' + q + contacts = F cos(omega_1 t) with a stop at q = gap (and at -gap)."""
    s = System("impact", np.eye(1), np.array([[c]]), np.eye(1), np.zeros((0, 3), np.int32), np.zeros(0),
               np.zeros((0, 4), np.int32), np.zeros(0), np.array([[F]]))
    if two_sided:
        return with_contacts(s, [0, 0], [1, -1], [gap, gap], [kc, kc])
    return with_contacts(s, [0], [1], [gap], [kc])

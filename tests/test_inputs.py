"""Pins of the synthetic system builders (inputs shared by oracle and HIP tests)."""
import os

import numpy as np
import pytest

from fse_inputs import cantilever_hermite_beam, synthetic_shell, vk_beam_clamped
from fse_inputs.systems import natural_frequencies

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_cantilever_first_frequency():
    """Euler-Bernoulli cantilever: omega_1 = 1.8751^2 sqrt(EI / (rho A L^4))."""
    s = cantilever_hermite_beam()
    EI = 210e9 * 0.02 ** 4 / 12
    w1 = 1.87510407 ** 2 * np.sqrt(EI / (7800 * 4e-4))
    assert s.n == 10
    assert abs(natural_frequencies(s.M, s.K, 1)[0] / w1 - 1) < 2e-4


def test_vk_beam_first_frequency_and_load_dof():
    """Clamped-clamped beam of Table 1: omega_1 = 4.7300^2 sqrt(EI/(rho A L^4)) = 44.55 rad/s,
    the neighbourhood of the paper's sweep (omega_1 = 44.5 ... 45.1, Sec. 4.1.1)."""
    s = vk_beam_clamped()
    EI = 45e9 * 0.01 ** 4 / 12
    w1 = 4.73004074 ** 2 * np.sqrt(EI / (1780 * 1e-4 * 2.7 ** 4))
    assert s.n == 147
    assert abs(natural_frequencies(s.M, s.K, 1)[0] / w1 - 1) < 2e-4
    # load at DOF 3 N_n / 2 - 1 (1-based) = midspan transverse DOF
    assert np.flatnonzero(s.F[0]).tolist() == [73]
    # von Karman tangent is symmetric (potential forces)
    from oracle.newmark import tangent
    q = np.random.default_rng(0).normal(size=147) * 1e-2
    Kt = tangent(s, q)
    assert np.allclose(Kt, Kt.T, atol=1e-9 * np.abs(Kt).max())


def test_shell_dof_counts_match_printed():
    rows = [tuple(int(v) for v in l.split()) for l in open(os.path.join(GOLD, "shell_dofs.txt"))
            if l.strip() and not l.startswith("#")]
    for NH, NL, dofs in rows:
        assert 6 * (NH + 1) * NL == dofs
    for NH, NL, dofs in rows[:2]:
        s = synthetic_shell(NH=NH, NL=NL)
        assert s.n == dofs
        assert abs(natural_frequencies(s.M, s.K, 1)[0] / (2 * np.pi * 100) - 1) < 1e-9

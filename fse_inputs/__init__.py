"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package builds the *system model* only: finite-element matrices M, D, K,
sparse polynomial internal-force tensors, load vectors, torus discretisation
parameters and initial iterates.  It contains none of the FSE-Shooting
arithmetic (no Fourier matrices, no time integration, no shooting residual),
so the CPU oracle and the HIP path can both consume it without sharing code.
"""
from .systems import (System, Torus, Workload, cantilever_hermite_beam,
                      vk_beam_clamped, synthetic_shell, tiny_system,
                      linear_oscillator, workload)

__all__ = ["System", "Torus", "Workload", "cantilever_hermite_beam",
           "vk_beam_clamped", "synthetic_shell", "tiny_system",
           "linear_oscillator", "workload"]

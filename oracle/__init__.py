"""FP64 CPU oracle of FSE-Shooting — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct numpy implementation of what the HIP path
computes, written from the paper's equations (Sec. 3, Apps. B-F).  It shares no
code with the HIP library and neither imports the other.  Only `tests/`,
`__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py` may import
it; the product path never routes through it.

Modules
  torus     harmonic table (App. B), sample grid (Eq. D1), Gamma / Gamma^-1
            (Eqs. D2-D3), phase-shift rotation R(rho) (Eq. 14), nabla (Eq. 19),
            dR/domega (Eq. 24)
  newmark   per-trajectory average-acceleration Newmark with per-step Newton
            (Eqs. E2-E7) and exact discrete sensitivities (Eqs. E8-E9)
  shooting  AFT pipeline, shooting residual (Eqs. 15-16, 20-21), Jacobian
            (Eqs. 22-24), bordered Newton step (Sec. 3.2, Eqs. 17-18)
  lyapunov  Lyapunov exponents from the shooting by-product (App. F)
  learned   secant predictor, snapshot POD, MLP forward/backward (FP64)

Parity status of every function is listed in its module header.
"""

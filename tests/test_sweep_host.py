"""Host logic of the shell sweep in bench.py (no GPU): the sweep's point layout and the
control flow of its Newton-Krylov solver with Jacobian reuse, driven by a scripted stand-in for
the library whose residual falls by a fixed factor per step.

The stand-in's state is one number, the error e of the iterate: ||R|| = |e| + floor; a chord
step multiplies e by its rate, a full Newton step by 1e-3.  Checked: the returned iterate is the
first one below the tolerance; a refresh follows a step that contracts less than 4x, after a
check of ||R|| from the states alone, and is skipped when that check has converged; a step that
makes no progress is redone as a full step from the best iterate; a floor above the tolerance
ends the point as not converged at its best iterate, within a bounded number of steps."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

bench.progress = lambda msg: None


class _Z:
    def __init__(self, e=0.0):
        self.e = e

    def copy_(self, other):
        self.e = other.e
        return self

    def __getitem__(self, key):
        return self


class _Torch:
    @staticmethod
    def empty_like(z):
        return _Z()


def _lib(floor=0.0, chord=0.2, worse_below=None):
    calls = []

    def resid(z):
        return abs(z.e) + floor

    class Lib:
        @staticmethod
        def fse_newton_krylov_step(ctx, om, Z, **kw):
            r = resid(Z)
            Z.e *= 1e-3
            calls.append(("full", r))
            return r, 2, 0.0

        @staticmethod
        def fse_newton_krylov_chord_step(ctx, om, Z, **kw):
            r = resid(Z)
            Z.e *= 1.05 if (worse_below is not None and abs(Z.e) < worse_below) else chord
            calls.append(("chord", r))
            return r, 2, 0.0

        @staticmethod
        def fse_shooting_residual_jacobian(ctx, om, Z):
            calls.append(("check", resid(Z)))
            return None, np.array([resid(Z)]), None

    return Lib, calls


def _solve(lib, e0, have_J=True):
    Z = _Z(e0)
    out = bench.chord_solve(lib, _Torch, None, np.array([1.0, 2.0]), Z, {"have_J": have_J})
    return out, Z


def test_chord_steps_converge_and_return_the_first_converged_iterate():
    lib, calls = _lib(chord=0.2)
    (its, full, rn, ok), Z = _solve(lib, 1e-5)
    assert ok and full == 0 and [k for k, _ in calls] == ["chord"] * 6
    assert rn < bench.SWEEP_TOL and abs(Z.e) == rn
    assert its == 5


def test_slow_contraction_refreshes_after_a_state_only_check():
    lib, calls = _lib(chord=0.3)
    (its, full, rn, ok), Z = _solve(lib, 1e-5)
    kinds = [k for k, _ in calls]
    assert ok and full == 1
    assert kinds == ["chord", "chord", "check", "full", "check"]
    assert rn < bench.SWEEP_TOL


def test_first_point_without_a_stored_jacobian_starts_with_a_full_step():
    lib, calls = _lib(chord=0.2)
    (its, full, rn, ok), Z = _solve(lib, 1e-5, have_J=False)
    assert ok and calls[0][0] == "full"


def test_a_step_that_makes_things_worse_is_redone_from_the_best_iterate():
    lib, calls = _lib(chord=0.2, worse_below=3e-8)
    (its, full, rn, ok), Z = _solve(lib, 1e-5)
    kinds = [k for k, _ in calls]
    assert ok and full == 1 and rn < bench.SWEEP_TOL
    # the full step starts from the best iterate (1.6e-8), not from the worse one (1.68e-8)
    i = kinds.index("full")
    assert abs(calls[i][1] - 1.6e-8) < 1e-20


def test_a_floor_above_the_tolerance_ends_as_not_converged():
    lib, calls = _lib(floor=1.2e-8, chord=0.2)
    (its, full, rn, ok), Z = _solve(lib, 1e-5)
    assert not ok
    assert len(calls) < 20
    assert abs(rn - (abs(Z.e) + 1.2e-8)) < 1e-20          # Z is the best iterate, rn its residual


def test_sweep_points_interleave_inside_the_box():
    train, evalp = bench.sweep_points()
    assert train.shape == (100, 2) and evalp.shape == (100, 2)
    lo = np.array([bench.SWEEP_W[0], bench.SWEEP_A[0]])
    hi = np.array([bench.SWEEP_W[1], bench.SWEEP_A[1]])
    assert np.all(train >= lo - 1e-12) and np.all(train <= hi + 1e-12)
    assert np.all(evalp > lo) and np.all(evalp < hi)
    # no evaluation point is a training point, and consecutive points are grid neighbours
    d = np.abs(evalp[:, None, :] - train[None, :, :]).sum(-1)
    assert d.min() > 1e-6
    step = (hi - lo) / 9.0
    for pts in (train, evalp):
        jumps = np.abs(np.diff(pts, axis=0)) / step
        assert np.all(jumps.max(axis=1) <= 1.0 + 1e-9)
    # evaluation starts next to where training ends
    assert np.all(np.abs(evalp[0] - train[-1]) / step < 1.0)

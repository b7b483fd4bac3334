"""Host-side argument checks of the Python binding (no GPU: nothing is launched)."""
import numpy as np
import pytest

import paper_2508_06302_amd as fse


def test_unknown_frequency_calls_need_a_writable_float64_omega():
    """With d > e the updated frequencies are written back into omega; a list, a float32 array
    or a non-contiguous view would silently lose them, so they are refused before any call."""
    good = np.array([1.0, 2.0])
    assert np.array_equal(fse._omega_inout(good, 2, 1), good)
    for bad in ([1.0, 2.0], np.array([1.0, 2.0], np.float32), np.array([1.0, 0.0, 2.0, 0.0])[::2]):
        with pytest.raises(TypeError):
            fse._omega_inout(bad, 2, 1)
    ro = np.array([1.0, 2.0])
    ro.flags.writeable = False
    with pytest.raises(TypeError):
        fse._omega_inout(ro, 2, 1)
    # d = e: omega is only read, anything array-like is accepted
    assert np.array_equal(fse._omega_inout([1.0, 2.0], 2, 2), good)
    out = np.zeros(2)
    fse._omega_back(out, np.array([3.0, 4.0]))
    assert np.array_equal(out, [3.0, 4.0])

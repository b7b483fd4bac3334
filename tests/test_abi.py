"""The C-ABI library loads and exports every entry point declared in include/fse.h (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fse.h")
LIB = os.path.join(ROOT, "paper_2508_06302_amd", "libfse.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fse_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_five_named_calls():
    names = declared()
    for n in ("fse_init_torus", "fse_integrate_batch", "fse_shooting_residual_jacobian",
              "fse_newton_step", "fse_lyapunov"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfse.so not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (bind to torch's HIP runtime, as the binding does)
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfse.so not built")
def test_binding_declares_every_export():
    from paper_2508_06302_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()
    _lib.load()

"""Machine-code checks of the LDS-heavy trajectory kernels (host compile only, no GPU).

The fused trajectory kernel and the omega_1 sensitivity kernels keep their banded factors and
tensors in LDS, the wide-band kernels stage state rows, factor rings and operand blocks there,
and the dense LU stages its panels, triangles and permutations there (in FP64 and FP32).  Every LDS access must compile to a ds_* instruction: a generic (flat) access to
LDS with a 16-byte load at an 8-byte-aligned address is the code-generation outcome that lined
up with the memory-aperture faults the fused kernel once had, and typing every pointer with its
address space removed it.  This test fails if any flat memory instruction reappears in those
units' gfx950 code."""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2508_06302_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
UNITS = ["k_fused.hip", "k_wsens.hip", "k_wide.hip", "k_linalg.hip"]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_lds_kernels_have_no_flat_memory_instructions():
    with tempfile.TemporaryDirectory() as tmp:
        procs = []
        for u in UNITS:
            out = os.path.join(tmp, u + ".s")
            cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                   "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", "-o", out,
                   os.path.join(SRC, u)]
            procs.append((u, out, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE)))
        for u, out, p in procs:
            _, err = p.communicate(timeout=600)
            assert p.returncode == 0, err.decode()[-2000:]
            asm = open(out).read()
            flat = re.findall(r"^\s+(flat_\w+)", asm, re.M)
            assert not flat, f"{u}: {len(flat)} flat memory instructions, e.g. {sorted(set(flat))[:4]}"
            assert re.search(r"^\s+ds_read", asm, re.M), f"{u}: no LDS reads found (check the compile)"

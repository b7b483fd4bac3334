"""Host arithmetic of bench.py's roofline (no GPU).

The wide-band sweep's algorithmic FP64 work per trajectory-step is 2n (2n + 2 nnz(D) + 4 nnz(L) + 6n):
the right-hand side (lumped M, sparse D), forward and backward substitution with the banded unit
factor, the pivot scaling and the updates.  Pinned against a count made here from the shell's matrices
(nnz(D) off the matrix, nnz(L) = n bw - bw (bw + 1) / 2 of a full band).  The HBM traffic of the profiled
kernel is used only while the stored summary was taken on the current kernel source."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_sweep_flops_per_trajectory_step_on_the_shell():
    from fse_inputs import workload
    s = workload("C3").system
    n = s.n
    D = np.asarray(s.D)
    rows, cols = np.nonzero(D)
    bw = int(np.max(np.abs(rows - cols)))
    nnz_d = rows.size
    nnz_l = sum(min(bw, n - 1 - j) for j in range(n))          # strictly lower band entries
    expect = 2 * n * (2 * n + 2 * nnz_d + 4 * nnz_l + n + 5 * n)
    assert (n, bw) == (1872, 89)
    assert bench.sweep_flops_per_traj_step(s, bw) == expect
    assert abs(expect - 3.04e9) < 0.01e9


def test_traffic_summary_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    current = {"source_sha256_16": bench.source_hash(["k_wide.hip"]), "bytes_per_launch": 1.5e10}
    stale = {"source_sha256_16": "0" * 16, "bytes_per_launch": 1.5e10}
    (tmp_path / "profiles" / "current.json").write_text(json.dumps(current))
    (tmp_path / "profiles" / "stale.json").write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("current.json", ["k_wide.hip"]) == 1.5e10
    assert bench.read_traffic("stale.json", ["k_wide.hip"]) is None
    assert bench.read_traffic("missing.json", ["k_wide.hip"]) is None

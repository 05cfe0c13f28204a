"""Host logic of bench.py, without a GPU: the algorithmic byte models, the guard that drops
measured traffic once the kernel source changes, and the refusal to run on several GPUs."""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_step_bytes_model():
    """matrix once (values + int32 columns + int64 row pointers) and three d x M vectors."""
    d, nnz, M = 1_000_000, 10_999_972, 64
    want = nnz * (4 + 4) + (d + 1) * 8 + 3 * d * M * 4
    assert bench.step_bytes(d, nnz, M, 4, 4) == want
    assert abs(want / 1e9 - 0.864) < 1e-3
    assert bench.step_bytes(10, 20, 3, 2, 8) == 20 * 6 + 11 * 8 + 3 * 10 * 3 * 8


def test_adjoint_bytes_model():
    d, nnz, M = 1_000_000, 10_999_972, 64
    pair = bench.adjoint_bytes(d, nnz, M, 4, 4, 4, True)
    plain = bench.adjoint_bytes(d, nnz, M, 4, 4, 4, False)
    assert pair - plain == 2 * d * M * 4  # the seed's W_(j-1) and W_(j+1)
    assert abs(pair / 1e9 - 1.72) < 1e-2


def test_traffic_needs_the_profiled_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1")
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = hashlib.sha256(b"kernel v1").hexdigest()
    (prof / "counters_step_toy.md").write_text(f"traffic_bytes_per_launch: 1.5e+09\nkernel_source_sha256: {sha}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    assert bench.traffic_from_profiles("step", "toy") == 1.5e9
    assert bench.traffic_from_profiles("adjoint", "toy") is None
    src.write_text("kernel v2")
    assert bench.traffic_from_profiles("step", "toy") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr

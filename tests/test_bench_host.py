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
    """The compulsory per-step count: matrix once (values + int32 columns + 4-byte row pointers) and
    three d x M vectors.  On the 4096^2 grid with BF16 values, M = 32: 7.01 GB per step."""
    d, nnz, M = 4096 * 4096, 83_869_696, 32
    want = nnz * (2 + 4) + (d + 1) * 4 + 3 * d * M * 4
    assert bench.step_bytes(d, nnz, M, 2, 4) == want
    assert abs(want / 1e9 - 7.012) < 1e-3
    assert bench.step_bytes(10, 20, 3, 2, 8) == 20 * 6 + 11 * 4 + 3 * 10 * 3 * 8


def test_adjoint_bytes_model():
    """The method's own adjoint work per step: the SpMM (matrix, y_(j+1) once, y_(j+2) read, y_j
    written), w_j read once, and 2 x 4 bytes of FP32 gradient accumulator per stored entry.  At
    random1m (d = 1e6, 10,999,972 entries, M = 64, FP32) that is 0.860 + 0.256 + 0.088 = 1.204 GB;
    the paired kernel also reads w_(j-1), w_(j+1) and int64 row pointers."""
    d, nnz, M = 1_000_000, 10_999_972, 64
    alg = bench.adjoint_bytes(d, nnz, M, 4, 4, 4)
    assert abs(alg / 1e9 - 1.204) < 1e-3
    assert alg == (nnz * 8 + (d + 1) * 4 + 3 * d * M * 4) + d * M * 4 + 8 * nnz
    moved = bench.adjoint_moved_bytes(d, nnz, M, 4, 4, 4, "explicit_single")
    assert moved - alg == 2 * d * M * 4 + (d + 1) * 4
    # the shifted form moves no extra vector block, only the int64 row pointers' extra half
    assert bench.adjoint_moved_bytes(d, nnz, M, 4, 4, 4, "shifted") - alg == (d + 1) * 4
    # staged stencil tiles: packed entries (8 bytes with FP32 values) in place of the CSR matrix
    staged = bench.adjoint_moved_bytes(d, nnz, M, 4, 4, 4, "shifted_staged")
    assert staged == alg - (nnz * 8 + (d + 1) * 4) + nnz * 8


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

"""GPU parity of the Taylor-series comparator (Section 5.1's accuracy comparison) with the oracle,
and the comparison itself on a grid with a closed-form log det."""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from tests._gpu import U32, U64, dev, floor_taylor, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ld():
    import torch

    assert torch.cuda.is_available()
    import paper_1503_06394_amd as pkg

    pkg.lib()
    return pkg


CASES = [
    ("grid32_f64", lambda: synth.grid_laplacian_2d(32, "f64"), 0.1, 30, 50, 1e-10),
    ("random1e4_f32", lambda: synth.random_sparse_spd(10_000, 5, 3, 1.0, "f32"), 0.0, 40, 64, 1e-4),
    ("random3001_f64_ragged", lambda: synth.random_sparse_spd(3001, 4, 5, 1.0, "f64"), 0.0, 17, 37, 1e-10),
    ("grid100_bf16_shift", lambda: synth.grid_laplacian_2d(100, "bf16"), 0.05, 25, 32, 1e-4),
]


@pytest.mark.parametrize("name,make,shift,n,M,tol", CASES, ids=[c[0] for c in CASES])
def test_taylor_parity(ld, oracle_lib, name, make, shift, n, M, tol):
    B = make()
    a, b = oracle_lib.gershgorin(B, shift)
    say(f"taylor {name} d={B.d} n={n} M={M}")
    r = ld.ld_logdet_taylor(dev(B, shift=shift), a, b, n, M, 7, want_probes=True, want_moments=True)
    o = oracle_lib.logdet_taylor(B, a, b, n, M, seed=7, shift=shift)
    assert rel(r["logdet"], o["gamma"], floor_taylor(a, b, n, B.d, tol, U64 if tol < 1e-6 else U32)) <= tol
    for j in range(M):
        assert rel(r["s"][j], o["s"][j], floor_taylor(a, b, n, B.d, tol, U64 if tol < 1e-6 else U32)) <= tol, j
    assert np.all(r["moments"][:, 0] == B.d)
    assert np.all(np.abs(r["moments"]) <= B.d * (1 + 1e-6))


@pytest.mark.parametrize("storage,M", [("bf16", 32), ("f32", 16)])
def test_taylor_staged_steps(ld, oracle_lib, storage, M, monkeypatch):
    """On a grid (a stencil pattern) with FP32 vectors every Taylor step reads W_k's rows from LDS
    tiles (the first from the probe hash): per-probe parity with the oracle and with the general step
    kernel (LD_STENCIL=0)."""
    monkeypatch.delenv("LD_STENCIL", raising=False)
    B = synth.grid_laplacian_2d(100, storage)
    shift, n = 0.05, 25
    a, b = oracle_lib.gershgorin(B, shift)
    D = dev(B, shift=shift)
    say(f"taylor staged {storage} M={M}")
    r = ld.ld_logdet_taylor(D, a, b, n, M, 7, want_probes=True)
    assert r["staged_steps"] == n, r["staged_steps"]
    o = oracle_lib.logdet_taylor(B, a, b, n, M, seed=7, shift=shift)
    fl = floor_taylor(a, b, n, B.d, 1e-4, U32)
    assert rel(r["logdet"], o["gamma"], fl) <= 1e-4
    for j in range(M):
        assert rel(r["s"][j], o["s"][j], fl) <= 1e-4, j
    monkeypatch.setenv("LD_STENCIL", "0")
    r0 = ld.ld_logdet_taylor(D, a, b, n, M, 7)
    assert r0["staged_steps"] == 0
    assert rel(r["logdet"], r0["logdet"], fl) <= 1e-4


@pytest.mark.parametrize("n", [0, 1, 2])
def test_taylor_low_degree(ld, oracle_lib, n):
    B = synth.random_sparse_spd(2000, 3, 8, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B)
    say(f"taylor low degree n={n}")
    r = ld.ld_logdet_taylor(dev(B), a, b, n, 8, 3)
    o = oracle_lib.logdet_taylor(B, a, b, n, 8, seed=3)
    if n == 0:
        assert r["logdet"] == B.d * math.log(a + b)
    assert rel(r["logdet"], o["gamma"], floor_taylor(a, b, n, B.d, 1e-12)) <= 1e-12


def test_chebyshev_beats_taylor_on_grid(ld):
    """Section 5.1's accuracy comparison: 256 x 256 Dirichlet grid + 0.1 I (closed-form log det),
    FP64, the same 64 probes and degree 30 for both estimators."""
    N = 256
    B = synth.grid_laplacian_2d(N, "f64")
    t = np.pi * np.arange(1, N + 1) / (N + 1)
    exact = float(np.log((4.0 - 2.0 * np.cos(t)[:, None] - 2.0 * np.cos(t)[None, :]) + 0.1).sum())
    D = dev(B, shift=0.1)
    say("taylor vs chebyshev on grid256")
    ch = ld.ld_logdet_cheb(D, 0.1, 8.1, 30, 64, 11)
    ta = ld.ld_logdet_taylor(D, 0.1, 8.1, 30, 64, 11)
    assert abs(ch["logdet"] - exact) < 0.1 * abs(ta["logdet"] - exact)
    assert abs(ta["logdet"] - exact) <= ta["poly_bound"] + 6 * ta["std_err"]

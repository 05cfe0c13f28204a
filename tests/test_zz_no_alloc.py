"""The forward entry point that allocates nothing (ld_logdet_cheb_noalloc), called through the C ABI,
against ld_logdet_cheb on the same inputs: two calls in a row on the shared scratch array, the second
on a smaller matrix, each at the parity tolerance of its precision (1e-10 FP64, 1e-4 FP32/BF16 on
the estimate, the per-probe estimates and the moments).  A problem beyond the array's size is refused
before any work and the array still serves the next call."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests._gpu import U32, U64, dev, floor_for, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ld():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1503_06394_amd as pkg

    pkg.lib()
    return pkg


def _agree(x, y, tol, a, b, n, d, u):
    fl = floor_for(a, b, n, d, tol, u)
    assert rel(x["logdet"], y["logdet"], fl) <= tol, (x["logdet"], y["logdet"])
    assert np.max(np.abs(x["s"] - y["s"])) <= tol * max(float(np.max(np.abs(y["s"]))), fl)
    assert np.max(np.abs(x["moments"] - y["moments"])) <= tol * d


def test_noalloc_matches_the_allocating_entry_point(ld):
    # first call: random sparse SPD, d = 100,000, FP32 values, M = 32, n = 30 (about 26 MB of scratch)
    B1 = synth.random_sparse_spd(100_000, 5, 7, 1.0, "f32")
    D1 = dev(B1)
    a1, b1 = ld.ld_gershgorin(D1)
    say("noalloc: random d=100000 FP32 M=32 n=30")
    x1 = ld.ld_logdet_cheb_noalloc(D1, a1, b1, 30, 32, 11, want_moments=True, want_probes=True)
    y1 = ld.ld_logdet_cheb(D1, a1, b1, 30, 32, 11, want_moments=True, want_probes=True)
    _agree(x1, y1, 1e-4, a1, b1, 30, B1.d, U32)
    # second call, smaller: 32 x 32 grid + 0.1 I, FP64, M = 50, n = 31 (odd degree, ragged last step)
    B2 = synth.grid_laplacian_2d(32, "f64")
    D2 = dev(B2, shift=0.1)
    say("noalloc: grid 32x32 FP64 M=50 n=31")
    x2 = ld.ld_logdet_cheb_noalloc(D2, 0.1, 8.1, 31, 50, 1, want_moments=True, want_probes=True)
    y2 = ld.ld_logdet_cheb(D2, 0.1, 8.1, 31, 50, 1, want_moments=True, want_probes=True)
    _agree(x2, y2, 1e-10, 0.1, 8.1, 31, B2.d, U64)
    # the same first problem again: the array holds the second call's contents, nothing carries over
    say("noalloc: random d=100000 again")
    x3 = ld.ld_logdet_cheb_noalloc(D1, a1, b1, 30, 32, 11, want_moments=True, want_probes=True)
    assert x3["logdet"] == x1["logdet"] and np.array_equal(x3["moments"], x1["moments"])


def test_noalloc_refuses_what_does_not_fit(ld):
    # d = 1,000,000 with M = 64 FP32 needs two 256 MB blocks: refused on the host
    B = synth.random_sparse_spd(1_000_000, 2, 3, 1.0, "f32")
    D = dev(B)
    a, b = ld.ld_gershgorin(D)
    say("noalloc: too large, refused")
    with pytest.raises(ld.LogdetChebError, match="scratch"):
        ld.ld_logdet_cheb_noalloc(D, a, b, 10, 64, 1)
    # a small problem right after still runs
    B2 = synth.grid_laplacian_2d(16, "f64")
    D2 = dev(B2, shift=0.5)
    say("noalloc: small after refusal")
    x = ld.ld_logdet_cheb_noalloc(D2, 0.5, 8.5, 12, 8, 3, want_moments=True, want_probes=True)
    y = ld.ld_logdet_cheb(D2, 0.5, 8.5, 12, 8, 3, want_moments=True, want_probes=True)
    _agree(x, y, 1e-10, 0.5, 8.5, 12, B2.d, U64)

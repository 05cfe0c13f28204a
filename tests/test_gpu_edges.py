"""Edge cases of every estimator entry point: the empty matrix, the largest probe block, very high
degree, and argument errors raised before any kernel runs."""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from tests._gpu import U32, U64, dev, floor_for, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ld():
    import torch

    assert torch.cuda.is_available()
    import paper_1503_06394_amd as pkg

    pkg.lib()
    return pkg


def _empty(ld, dtype):
    import torch

    return ld.DeviceCSR(torch.zeros(1, dtype=torch.int64, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"),
                        torch.zeros(0, dtype=dtype, device="cuda"))


@pytest.mark.parametrize("f64", [False, True])
def test_empty_matrix_has_log_det_zero(ld, f64):
    import torch

    E = _empty(ld, torch.float64 if f64 else torch.float32)
    say(f"empty matrix f64={f64}")
    for r in (ld.ld_logdet_cheb(E, 1.0, 2.0, 10, 4, 1, want_probes=True),
              ld.ld_logdet_cheb(E, 1.0, 2.0, 10, 4, 1, plain=True),
              ld.ld_logabsdet_cheb(E, None, 1.0, 2.0, 10, 4, 1),
              ld.ld_logdet_taylor(E, 1.0, 2.0, 10, 4, 1)):
        assert r["status"] == 0 and r["logdet"] == 0.0
    r, g = ld.ld_logdet_cheb_grad(E, 1.0, 2.0, 10, 4, 1)
    assert r["logdet"] == 0.0 and g.numel() == 0 and r["grad_shift"] == 0.0


def test_largest_probe_block(ld, oracle_lib):
    """M = 4096, the most one call accepts (many probe tiles per pass), FP32; M = 4097 is refused."""
    B = synth.random_sparse_spd(300, 3, 13, 1.0, "f32")
    a, b = oracle_lib.gershgorin(B)
    say("M = 4096")
    r = ld.ld_logdet_cheb(dev(B), a, b, 12, 4096, 5, want_probes=True)
    o = oracle_lib.logdet(B, a, b, 12, 4096, seed=5)
    fl = floor_for(a, b, 12, B.d, 1e-4, U32)
    assert rel(r["logdet"], o["gamma"], fl) <= 1e-4
    for j in (0, 63, 64, 2047, 4095):
        assert rel(r["s"][j], o["s"][j], fl) <= 1e-4, j
    with pytest.raises(ld.LogdetChebError):
        ld.ld_logdet_cheb(dev(B), a, b, 12, 4097, 5)


@pytest.mark.parametrize("plain", [False, True])
def test_high_degree_fp64(ld, oracle_lib, plain):
    """n = 2000 (the recurrence and the product identities stay within FP64 parity)."""
    B = synth.random_sparse_spd(400, 3, 17, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B)
    say(f"n = 2000 plain={plain}")
    r = ld.ld_logdet_cheb(dev(B), a, b, 2000, 8, 6, plain=plain)
    o = oracle_lib.logdet(B, a, b, 2000, 8, seed=6)
    assert rel(r["logdet"], o["gamma"], floor_for(a, b, 2000, B.d, 1e-10, U64)) <= 1e-10


def test_argument_errors_before_any_kernel(ld):
    B = dev(synth.random_sparse_spd(100, 3, 2, 1.0, "f32"))
    say("argument errors")
    bad = [(0.0, 1.0, 10, 4), (2.0, 1.0, 10, 4), (1.0, 1.0, 10, 4), (float("nan"), 2.0, 10, 4),
           (1.0, float("inf"), 10, 4), (1.0, 2.0, -1, 4), (1.0, 2.0, 100001, 4), (1.0, 2.0, 10, 0)]
    for a, b, n, M in bad:
        for f in (ld.ld_logdet_cheb, ld.ld_logdet_taylor):
            with pytest.raises(ld.LogdetChebError):
                f(B, a, b, n, M, 1)
        with pytest.raises(ld.LogdetChebError):
            ld.ld_logdet_cheb_grad(B, a, b, n, M, 1)
    with pytest.raises(ld.LogdetChebError):
        ld.ld_logabsdet_cheb(B, None, 0.0, 1.0, 10, 4, 1)
    shifted = ld.DeviceCSR(B.row_ptr, B.col, B.values, 0.5)
    with pytest.raises(ld.LogdetChebError, match="diag_shift"):
        ld.ld_logabsdet_cheb(shifted, None, 0.5, 1.0, 10, 4, 1)


def _graph_laplacian_plus_identity(G):
    """L + I of a graph: -1 per edge, degree + 1 on the diagonal (rows sorted by column)."""
    rows = np.repeat(np.arange(G.d), np.diff(G.row_ptr))
    r = np.concatenate([rows, np.arange(G.d)])
    c = np.concatenate([G.col.astype(np.int64), np.arange(G.d)])
    v = np.concatenate([-np.ones(G.nnz), np.diff(G.row_ptr) + 1.0])
    o = np.lexsort((c, r))
    row_ptr = np.zeros(G.d + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=G.d), out=row_ptr[1:])
    return synth.CSR(G.d, row_ptr, c[o].astype(np.int32), v[o], "f64", {})


@pytest.mark.parametrize("plain", [False, True])
def test_row_longer_than_the_lds_slice(ld, oracle_lib, plain):
    """A hub row with 4999 stored entries overflows the LDS staging of its tile, which then reads
    the CSR from global memory: forward and gradient against the oracle (FP64)."""
    B = _graph_laplacian_plus_identity(synth.hub_graph(5000, 2, 3))
    assert np.diff(B.row_ptr).max() > 4096
    a, b = oracle_lib.gershgorin(B)
    say(f"long row: forward and gradient plain={plain}")
    r = ld.ld_logdet_cheb(dev(B), a, b, 20, 16, 4, plain=plain)
    o = oracle_lib.logdet(B, a, b, 20, 16, seed=4)
    assert rel(r["logdet"], o["gamma"], floor_for(a, b, 20, B.d, 1e-10, U64)) <= 1e-10
    rg, g = ld.ld_logdet_cheb_grad(dev(B), a, b, 20, 16, 4, plain=plain)
    og = oracle_lib.logdet_grad(B, a, b, 20, 16, seed=4)
    gg = g.cpu().numpy()
    assert np.max(np.abs(gg - og["grad"])) <= 1e-10 * np.max(np.abs(og["grad"]))


@pytest.mark.parametrize("nbytes", [1, 15, 16, 4096 * 16 + 7, (1 << 20) + 3, 64 << 20])
def test_copy_kernel_is_exact(ld, nbytes):
    """The streaming copy used as the bandwidth reference copies every byte, tails included."""
    import torch

    say(f"copy {nbytes} bytes")
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes + 32,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros(nbytes + 32, dtype=torch.uint8, device="cuda")
    ld.ld_copy(dst[:nbytes], src[:nbytes])
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].count_nonzero()) == 0


def test_degree_zero_gradient_is_zero(ld, oracle_lib):
    """At n = 0 the estimate d log((a+b)/2) does not depend on B: zero gradient, zero d/dshift."""
    B = synth.random_sparse_spd(500, 3, 23, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B)
    say("gradient at n = 0")
    r, g = ld.ld_logdet_cheb_grad(dev(B), a, b, 0, 8, 1)
    assert r["logdet"] == pytest.approx(B.d * math.log((a + b) / 2), rel=1e-15)
    assert float(g.abs().max()) == 0.0 and r["grad_shift"] == 0.0
    o = oracle_lib.logdet_grad(B, a, b, 0, 8, seed=1)
    assert np.all(o["grad"] == 0.0) and o["grad_shift"] == 0.0


def test_internal_workspaces_reused_across_sizes_threads_and_clears(ld):
    """Calls without a workspace of their own draw on the library's pooled buffers: results stay
    bit-identical across alternating sizes, concurrent calls from two threads on two streams, and
    ld_clear_cache."""
    import threading

    import torch

    mats = [synth.random_sparse_spd(d, 3, 30 + i, 1.0, "f32") for i, d in enumerate([700, 30_000, 5_000])]
    D = [dev(B) for B in mats]
    ab = [ld.ld_gershgorin(x) for x in D]
    say("pooled workspaces: reference results")
    ref = [ld.ld_logdet_cheb(D[i], *ab[i], 20, 16, 4)["logdet"] for i in range(3)]
    for _ in range(3):
        for i in (2, 0, 1):
            assert ld.ld_logdet_cheb(D[i], *ab[i], 20, 16, 4)["logdet"] == ref[i]
    ld.ld_clear_cache()
    assert [ld.ld_logdet_cheb(D[i], *ab[i], 20, 16, 4)["logdet"] for i in range(3)] == ref
    say("pooled workspaces: two threads")
    out = {}

    def work(tag, order, stream):
        with torch.cuda.stream(stream):
            out[tag] = [ld.ld_logdet_cheb(D[i], *ab[i], 20, 16, 4, stream=stream)["logdet"] for i in order * 4]

    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    t1 = threading.Thread(target=work, args=("a", [0, 1, 2], s1))
    t2 = threading.Thread(target=work, args=("b", [2, 1, 0], s2))
    t1.start(); t2.start(); t1.join(); t2.join()
    assert out["a"] == [ref[i] for i in [0, 1, 2] * 4]
    assert out["b"] == [ref[i] for i in [2, 1, 0] * 4]


@pytest.mark.parametrize("plain", [False, True])
def test_high_degree_fp32(ld, oracle_lib, plain):
    """n = 400 on the FP32 path: the product identities form mu_2k = 2 |W_k|^2 - d, a difference of
    O(d) terms; parity with the oracle must still hold at the FP32 tolerance."""
    B = synth.random_sparse_spd(20_000, 4, 27, 1.0, "f32")
    a, b = oracle_lib.gershgorin(B)
    say(f"n = 400 FP32 plain={plain}")
    r = ld.ld_logdet_cheb(dev(B), a, b, 400, 16, 8, plain=plain, want_probes=True)
    o = oracle_lib.logdet(B, a, b, 400, 16, seed=8)
    fl = floor_for(a, b, 400, B.d, 1e-4, U32)
    assert rel(r["logdet"], o["gamma"], fl) <= 1e-4
    for j in range(16):
        assert rel(r["s"][j], o["s"][j], fl) <= 1e-4, j

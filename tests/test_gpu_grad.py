"""GPU parity of the gradient (adjoint recurrence with checkpoints) against the oracle's reverse
mode, plus the torch.autograd wrapper and the GMRF chain rule through (tau, kappa)."""
from __future__ import annotations

import warnings

import numpy as np
import pytest

import synth
from tests._gpu import dev, entrywise, floor_for, rel, say
from tests._patterns import _banded, _grid2d_rect, _hex2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ld():
    import torch

    assert torch.cuda.is_available()
    import paper_1503_06394_amd as pkg

    pkg.lib()
    return pkg


# Adjoint forms: the product-identity form with the explicit seed (single gather per entry) or the
# shifted one (two gathers, two vector blocks less per step) on vector tiles staged in LDS or on
# global gathers, and the plain recurrence.
FORMS = ["explicit", "shifted", "shifted_global", "plain"]
# what may run: the shifted form runs on staged tiles where the pattern is a stencil pattern for the
# pass's tile, on global gathers elsewhere
RAN = {"explicit": ("explicit_single",), "shifted": ("shifted", "shifted_staged"), "shifted_global": ("shifted",),
       "plain": ("plain",)}


def _use_form(monkeypatch, form: str) -> bool:
    """Select the adjoint form; returns the `plain` argument."""
    monkeypatch.delenv("LD_STENCIL", raising=False)
    if form == "plain":
        monkeypatch.delenv("LD_GRAD_FORM", raising=False)
        return True
    if form == "shifted_global":
        monkeypatch.setenv("LD_STENCIL", "0")
        form = "shifted"
    monkeypatch.setenv("LD_GRAD_FORM", form)
    return False


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 30])
@pytest.mark.parametrize("stride", [0, 1, 2, 3, 5, 100])
def test_grad_fp64_parity(ld, oracle_lib, n, stride, form, monkeypatch):
    """Gradient along symmetric perturbations, per stored entry, against the oracle's reverse mode:
    both product-identity forms and the plain recurrence, every checkpoint stride."""
    plain = _use_form(monkeypatch, form)
    B = synth.random_sparse_spd(2000, 4, 17, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B)
    M, seed, shift, go = 16, 9, 0.25, 1.7
    say(f"grad fp64 n={n} stride={stride} form={form}")
    r, g = ld.ld_logdet_cheb_grad(dev(B, shift=shift), a + shift, b + shift, n, M, seed, go, ckpt_stride=stride,
                                  plain=plain)
    o = oracle_lib.logdet_grad(B, a + shift, b + shift, n, M, seed=seed, shift=shift)
    assert r["adjoint_form"] in RAN[form]
    assert entrywise(g.cpu().numpy(), go * o["grad"]) <= 1e-10
    assert rel(r["grad_shift"], go * o["grad_shift"]) <= 1e-10
    assert rel(r["logdet"], o["gamma"]) <= 1e-10


def test_grad_rows_without_diagonal(ld, oracle_lib):
    B = synth.random_sparse_spd(900, 3, 5, 1.0, "f64")
    rows = B.row_of_entry()
    keep = ~((rows % 2 == 0) & (B.col == rows))
    rp = np.zeros(B.d + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows[keep], minlength=B.d), out=rp[1:])
    C = synth.CSR(B.d, rp, B.col[keep], B.val[keep], "f64")
    shift = 12.0
    a, b = oracle_lib.gershgorin(C, shift)
    say("grad no-diagonal rows")
    r, g = ld.ld_logdet_cheb_grad(dev(C, shift=shift), a, b, 15, 8, 2)
    o = oracle_lib.logdet_grad(C, a, b, 15, 8, seed=2, shift=shift)
    assert entrywise(g.cpu().numpy(), o["grad"]) <= 1e-10
    assert rel(r["grad_shift"], o["grad_shift"]) <= 1e-10


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("M", [1, 3, 32, 64])
def test_grad_fp32_gmrf_parity(ld, oracle_lib, M, form, monkeypatch):
    """3-D GMRF precision Q = tau (kappa^2 I + L) in FP32 with the kappa^2 shift kept in FP64."""
    plain = _use_form(monkeypatch, form)
    N, tau, kappa, n = 10, 1.0, 0.3, 60
    L = synth.grid_laplacian_3d(N, "f32")
    shift = tau * kappa ** 2
    a, b = tau * kappa ** 2, tau * (kappa ** 2 + 12.0)
    say(f"grad fp32 gmrf M={M} form={form}")
    r, g = ld.ld_logdet_cheb_grad(dev(L, shift=shift), a, b, n, M, 3, plain=plain)
    assert r["adjoint_form"] in RAN[form]
    o = oracle_lib.logdet_grad(L, a, b, n, M, seed=3, shift=shift)
    assert entrywise(g.cpu().numpy(), o["grad"]) <= 1e-4
    assert rel(r["grad_shift"], o["grad_shift"]) <= 1e-4
    assert rel(r["logdet"], o["gamma"]) <= 1e-4


STENCIL_CASES = {
    # name: (builder, shift, M, degree, staged by default)
    "grid2d_ragged_f64": (lambda: _grid2d_rect(37, 41, "f64"), 0.3, 16, 24, True),
    "grid2d_f32_M32": (lambda: _grid2d_rect(64, 64, "f32"), 0.05, 32, 40, True),
    "grid2d_ragged_bf16_M32": (lambda: _grid2d_rect(45, 37, "bf16"), 0.05, 32, 30, True),  # the headline's types
    "grid2d_ragged_bf16_M18": (lambda: _grid2d_rect(29, 53, "bf16"), 0.2, 18, 25, True),  # 2 probes per lane
    "grid3d_f32_M64": (lambda: synth.grid_laplacian_3d(12, "f32"), 0.2, 64, 30, False),  # halo of 4 tiles
    "hex2d_f64_K7": (lambda: _hex2d(33, 29, "f64"), 0.1, 16, 22, True),
    "band3_f64_M8": (lambda: _banded(1500, 3, "f64", 4), 0.0, 8, 20, True),
    "grid2d_nodiag_f64": (lambda: _grid2d_rect(30, 33, "f64", drop_diag_every=3), 4.5, 16, 18, False),  # no diagonal
    "grid2d_passes_f32_M200": (lambda: _grid2d_rect(40, 40, "f32"), 0.1, 200, 16, True),
    "band5_k11_f64": (lambda: _banded(900, 5, "f64", 6), 0.0, 16, 14, False),  # 11 entries per row
}


@pytest.mark.parametrize("case", sorted(STENCIL_CASES))
def test_grad_stencil_patterns(ld, oracle_lib, case, monkeypatch):
    """Patterns whose tiles reach a fixed offset list (grids in natural order, bands): by default the
    shifted adjoint runs on vector tiles staged in LDS.  Entry by entry against the oracle, with
    ragged last tiles and several probe passes; rows without a stored diagonal and rows too long for
    the staged layout fall back to the explicit form."""
    monkeypatch.delenv("LD_GRAD_FORM", raising=False)
    monkeypatch.delenv("LD_STENCIL", raising=False)
    build, shift, M, n, staged = STENCIL_CASES[case]
    B = build()
    a, b = oracle_lib.gershgorin(B, shift)
    tol = 1e-10 if B.storage == "f64" else 1e-4
    say(f"grad stencil pattern {case} d={B.d} nnz={B.nnz} M={M} n={n}")
    r, g = ld.ld_logdet_cheb_grad(dev(B, shift=shift), a, b, n, M, 7)
    assert r["adjoint_form"] == ("shifted_staged" if staged else "explicit_single"), r["adjoint_form"]
    o = oracle_lib.logdet_grad(B, a, b, n, M, seed=7, shift=shift)
    assert entrywise(g.cpu().numpy(), o["grad"]) <= tol
    assert rel(r["grad_shift"], o["grad_shift"]) <= tol
    assert rel(r["logdet"], o["gamma"]) <= tol


def test_grad_stencil_repeat_bit_identical(ld, oracle_lib):
    """A second call on the same stencil pattern reuses the cached plan and its buffers and gives the
    same gradient bit for bit; another pattern in between does not disturb it."""
    import torch

    B = _grid2d_rect(50, 70, "f32")
    C = _banded(1200, 2, "f32", 9)
    DB, DC = dev(B, shift=0.2), dev(C)
    a, b = oracle_lib.gershgorin(B, 0.2)
    ac, bc = oracle_lib.gershgorin(C)
    say("grad stencil repeat")
    r1, g1 = ld.ld_logdet_cheb_grad(DB, a, b, 22, 32, 3)
    rc_, gc = ld.ld_logdet_cheb_grad(DC, ac, bc, 22, 32, 3)
    r2, g2 = ld.ld_logdet_cheb_grad(DB, a, b, 22, 32, 3)
    assert r1["adjoint_form"] == r2["adjoint_form"] == rc_["adjoint_form"] == "shifted_staged"
    assert torch.equal(g1, g2) and r1["logdet"] == r2["logdet"] and r1["grad_shift"] == r2["grad_shift"]


# 3-D lattices in natural order (neighbours at +-1, +-N, +-N^2): (N, storage, M, degree, tiles per plane)
PLANE_CASES = {
    "N16_f64_M16": (16, "f64", 16, 20, 8),
    "N16_f32_M32": (16, "f32", 32, 24, 8),
    "N32_f32_M32": (32, "f32", 32, 16, 32),
}


@pytest.mark.parametrize("case", sorted(PLANE_CASES))
def test_grad_plane_order(ld, oracle_lib, case, monkeypatch):
    """Plane-major tile order on 3-D lattices, forced at sizes where row order would be kept
    (LD_PLANE=1): entry by entry against the oracle, and bit for bit equal to the row-order call
    (LD_PLANE=0), since only the order in which the tiles run changes."""
    import torch

    monkeypatch.delenv("LD_GRAD_FORM", raising=False)
    monkeypatch.delenv("LD_STENCIL", raising=False)
    N, storage, M, n, per = PLANE_CASES[case]
    B = synth.grid_laplacian_3d(N, storage)
    shift = 0.15
    a, b = oracle_lib.gershgorin(B, shift)
    D = dev(B, shift=shift)
    say(f"grad plane order {case} d={B.d} nnz={B.nnz}")
    monkeypatch.setenv("LD_PLANE", "1")
    r1, g1 = ld.ld_logdet_cheb_grad(D, a, b, n, M, 5)
    assert r1["plane_tiles"] == per, r1["plane_tiles"]
    monkeypatch.setenv("LD_PLANE", "0")
    r0, g0 = ld.ld_logdet_cheb_grad(D, a, b, n, M, 5)
    assert r0["plane_tiles"] == 0
    assert torch.equal(g0, g1) and r0["logdet"] == r1["logdet"] and r0["grad_shift"] == r1["grad_shift"]
    monkeypatch.delenv("LD_PLANE")
    r2, _ = ld.ld_logdet_cheb_grad(D, a, b, n, M, 5)
    assert r2["plane_tiles"] == 0  # planes of N^2 rows too short to leave row order by default
    tol = 1e-10 if storage == "f64" else 1e-4
    o = oracle_lib.logdet_grad(B, a, b, n, M, seed=5, shift=shift)
    assert entrywise(g1.cpu().numpy(), o["grad"]) <= tol
    assert rel(r1["grad_shift"], o["grad_shift"]) <= tol
    assert rel(r1["logdet"], o["gamma"]) <= tol


def test_grad_plane_order_default_on_large_planes(ld, monkeypatch):
    """A 96^3 lattice with 32 FP32 probes (planes of 9216 rows, 1.1 MiB of vector rows) takes the
    plane-major order by default, 72 tiles of 128 rows per plane (the default row-order tile is 224
    rows), and gives the result of row order on the same 128-row tiles bit for bit.  A 12^3 lattice,
    whose +-N neighbours are too far from the diagonal relative to a plane, is not taken for one."""
    import torch

    monkeypatch.delenv("LD_GRAD_FORM", raising=False)
    monkeypatch.delenv("LD_STENCIL", raising=False)
    monkeypatch.delenv("LD_PLANE", raising=False)
    B = synth.grid_laplacian_3d(96, "f32")
    D = dev(B, shift=0.1)
    a, b = ld.ld_gershgorin(D)
    say(f"grad plane order default d={B.d}")
    r1, g1 = ld.ld_logdet_cheb_grad(D, a, b, 20, 32, 8)
    assert r1["plane_tiles"] == 72, r1["plane_tiles"]
    monkeypatch.setenv("LD_PLANE", "0")
    r0, g0 = ld.ld_logdet_cheb_grad(D, a, b, 20, 32, 8, tile=128)
    assert r0["plane_tiles"] == 0
    assert torch.equal(g0, g1) and r0["logdet"] == r1["logdet"] and r0["grad_shift"] == r1["grad_shift"]
    monkeypatch.setenv("LD_PLANE", "1")
    C = synth.grid_laplacian_3d(12, "f32")
    DC = dev(C, shift=0.1)
    ac, bc = ld.ld_gershgorin(DC)
    rc_, _ = ld.ld_logdet_cheb_grad(DC, ac, bc, 10, 32, 8)
    assert rc_["plane_tiles"] == 0


def _pattern_case(kind: str):
    """Symmetric matrices whose patterns stress the transpose lookup of the symmetric adjoint:
    a hub row joined to every vertex, rows left empty (carried by the diagonal shift alone), and
    rows whose columns are stored out of order."""
    rng = np.random.default_rng(61)
    if kind == "hub":
        G = synth.hub_graph(3000, 2, mseed=5)  # L + I of a graph with one vertex of degree 2999
        deg = np.diff(G.row_ptr).astype(np.float64)
        rp, col, val = synth._insert_diagonal(G.d, G.row_ptr, G.col, -G.val, deg)
        return synth.CSR(G.d, rp, col, val, "f64"), 1.0
    B = synth.random_sparse_spd(1500, 3, 31, 1.0, "f64")
    rows = B.row_of_entry()
    if kind == "empty_rows":
        gone = np.zeros(B.d, dtype=bool)
        gone[::7] = True
        keep = ~(gone[rows] | gone[B.col])
        rp = np.zeros(B.d + 1, dtype=np.int64)
        np.cumsum(np.bincount(rows[keep], minlength=B.d), out=rp[1:])
        return synth.CSR(B.d, rp, B.col[keep], B.val[keep], "f64"), 0.5
    order = np.concatenate([B.row_ptr[r] + rng.permutation(B.row_ptr[r + 1] - B.row_ptr[r])
                            for r in range(B.d)])
    return synth.CSR(B.d, B.row_ptr, B.col[order], B.val[order], "f64"), 0.0


@pytest.mark.parametrize("form", ["explicit", "shifted", "shifted_global"])
@pytest.mark.parametrize("kind", ["hub", "empty_rows", "unsorted"])
def test_grad_pattern_layouts(ld, oracle_lib, kind, form, monkeypatch):
    _use_form(monkeypatch, form)
    C, shift = _pattern_case(kind)
    a, b = oracle_lib.gershgorin(C, shift)
    say(f"grad pattern layout {kind} d={C.d} nnz={C.nnz} form={form}")
    r, g = ld.ld_logdet_cheb_grad(dev(C, shift=shift), a, b, 15, 8, 3)
    o = oracle_lib.logdet_grad(C, a, b, 15, 8, seed=3, shift=shift)
    assert entrywise(g.cpu().numpy(), o["grad"]) <= 1e-10
    assert rel(r["grad_shift"], o["grad_shift"]) <= 1e-10
    assert rel(r["logdet"], o["gamma"]) <= 1e-10


@pytest.mark.parametrize("storage,M", [("f32", 300), ("f32", 256), ("f64", 150), ("f64", 128)])
def test_grad_probe_passes(ld, oracle_lib, storage, M):
    """Probe blocks wider than one pass (128 FP32 / 64 FP64 probes): the passes' probes are
    probes probe0.. of the same seed, so value, per-entry gradient and d/d(shift) match the
    oracle's over all M probes."""
    B = synth.random_sparse_spd(1200, 3, 33, 1.0, storage)
    a, b = oracle_lib.gershgorin(B)
    tol = 1e-10 if storage == "f64" else 1e-4
    say(f"grad probe passes {storage} M={M}")
    r, g = ld.ld_logdet_cheb_grad(dev(B, shift=0.2), a + 0.2, b + 0.2, 14, M, 12)
    o = oracle_lib.logdet_grad(B, a + 0.2, b + 0.2, 14, M, seed=12, shift=0.2)
    assert entrywise(g.cpu().numpy(), o["grad"]) <= tol
    assert rel(r["grad_shift"], o["grad_shift"]) <= tol
    assert rel(r["logdet"], o["gamma"]) <= tol
    f = ld.ld_logdet_cheb(dev(B, shift=0.2), a + 0.2, b + 0.2, 14, M, 12)
    assert rel(r["logdet"], f["logdet"]) <= tol


def test_grad_rejects_too_many_probes(ld):
    B = synth.grid_laplacian_2d(8, "f32")
    with pytest.raises(ld.LogdetChebError):
        ld.ld_logdet_cheb_grad(dev(B, shift=0.1), 0.1, 8.1, 5, 4097, 0)


def test_autograd_function_and_gmrf_chain_rule(ld, oracle_lib):
    """LogdetCheb backward gives d/dvalues and d/dshift; the chain rule through Q = tau(kappa^2 I + L)
    gives dGamma/dtau = sum_t grad_t L_t + grad_shift kappa^2 and dGamma/dkappa = grad_shift 2 tau kappa."""
    import torch

    N, n, M, seed = 8, 40, 32, 5
    L = synth.grid_laplacian_3d(N, "f64")
    tau = torch.tensor(1.3, dtype=torch.float64, device="cuda", requires_grad=True)
    kappa = torch.tensor(0.4, dtype=torch.float64, device="cuda", requires_grad=True)
    Lv = torch.tensor(L.val, dtype=torch.float64, device="cuda")
    rp = torch.tensor(L.row_ptr, device="cuda")
    col = torch.tensor(L.col, device="cuda")
    a = float((tau * kappa ** 2).detach())
    b = float((tau * (kappa ** 2 + 12.0)).detach())
    say("autograd gmrf")
    vals = tau * Lv
    shift = tau * kappa ** 2
    out = ld.LogdetCheb.apply(vals, shift, rp, col, a, b, n, M, seed)
    out.backward()
    Q = synth.CSR(L.d, L.row_ptr, L.col, 1.3 * L.val)
    o = oracle_lib.logdet_grad(Q, a, b, n, M, seed=seed, shift=1.3 * 0.16)
    dtau = float((o["grad"] * L.val).sum() + o["grad_shift"] * 0.16)
    dkap = float(o["grad_shift"] * 2 * 1.3 * 0.4)
    assert rel(float(out.detach()), o["gamma"]) <= 1e-10
    assert rel(float(tau.grad), dtau) <= 1e-9
    assert rel(float(kappa.grad), dkap) <= 1e-9


def test_grad_two_gather_path_matches(ld, oracle_lib, monkeypatch):
    """LD_GRAD_SYM=0 forces the general (two-gather) adjoint with the explicit seed on a symmetric
    pattern."""
    B = synth.random_sparse_spd(1500, 4, 23, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B)
    monkeypatch.setenv("LD_GRAD_SYM", "0")
    monkeypatch.setenv("LD_GRAD_FORM", "explicit")
    say("grad two-gather path fp64")
    r, g = ld.ld_logdet_cheb_grad(dev(B, shift=0.1), a + 0.1, b + 0.1, 20, 12, 4)
    o = oracle_lib.logdet_grad(B, a + 0.1, b + 0.1, 20, 12, seed=4, shift=0.1)
    assert entrywise(g.cpu().numpy(), o["grad"]) <= 1e-10
    assert rel(r["grad_shift"], o["grad_shift"]) <= 1e-10


def test_grad_nonsymmetric_pattern(ld, oracle_lib):
    """A pattern without its transpose: the plain recurrence forward on B and the adjoint on B^T give
    dGamma/dB_ij for each stored entry on its own, the derivative the oracle's reverse mode computes
    (pinned on the CPU by central differences on a non-symmetric matrix)."""
    # real spectrum inside [a, b] (Algorithm 1's premise on the eigenvalues): the diagonal, in [10, 14]
    C = synth.lower_triangular_nonsymmetric(800, 3, 5)
    a, b = oracle_lib.gershgorin(C)
    assert 0 < a < 10 and 14 < b
    for storage, tol in (("f64", 1e-10), ("f32", 1e-4), ("bf16", 1e-4)):
        Cx = synth.CSR(C.d, C.row_ptr, C.col, synth.round_to(C.val, storage), storage)
        for stride in (0, 3):
            say(f"grad non-symmetric pattern {storage} stride={stride}")
            r, g = ld.ld_logdet_cheb_grad(dev(Cx, shift=0.3), a + 0.3, b + 0.3, 15, 8, 7, 1.3, ckpt_stride=stride)
            o = oracle_lib.logdet_grad(Cx, a + 0.3, b + 0.3, 15, 8, seed=7, shift=0.3)
            assert entrywise(g.cpu().numpy(), 1.3 * o["grad"]) <= tol
            assert rel(r["grad_shift"], 1.3 * o["grad_shift"]) <= tol
            assert rel(r["logdet"], o["gamma"]) <= tol


@pytest.mark.parametrize("M", [8, 200])
def test_grad_plain_on_nonsymmetric_values(ld, oracle_lib, M):
    """plain=True assumes no symmetry: on a symmetric pattern whose values are not symmetric, the
    adjoint runs on B^T (its values gathered through the transposed-entry index) and each entry
    gets its own derivative, as in the oracle; M = 200 takes two probe passes."""
    B = synth.random_sparse_spd(1500, 3, 19, 1.0, "f64")
    rng = np.random.default_rng(2)
    off = B.col != B.row_of_entry()
    val = B.val.copy()
    val[off] *= rng.uniform(0.5, 1.0, size=int(off.sum()))  # keeps the diagonal dominant: Gershgorin a > 0
    C = synth.CSR(B.d, B.row_ptr, B.col, val, "f64")
    a, b = oracle_lib.gershgorin(C, 0.2)
    say(f"grad plain, symmetric pattern with non-symmetric values, M={M}")
    r, g = ld.ld_logdet_cheb_grad(dev(C, shift=0.2), a, b, 12, M, 5, plain=True)
    o = oracle_lib.logdet_grad(C, a, b, 12, M, seed=5, shift=0.2)
    assert entrywise(g.cpu().numpy(), o["grad"]) <= 1e-10
    assert rel(r["grad_shift"], o["grad_shift"]) <= 1e-10
    assert rel(r["logdet"], o["gamma"]) <= 1e-10
    # the two orientations of a pair really differ here
    gt = g.cpu().numpy()
    perm = {(int(i), int(j)): t for t, (i, j) in enumerate(zip(C.row_of_entry(), C.col))}
    tr = np.array([perm[(int(j), int(i))] for i, j in zip(C.row_of_entry(), C.col)])
    assert np.max(np.abs(gt - gt[tr])) > 1e-3 * np.max(np.abs(gt))


def test_grad_pattern_analysis_cached_and_rechecked(ld, oracle_lib):
    """The pattern's analysis is made once and reused: a second call matches the first bit for bit.
    Rewriting the pattern in place (same device arrays, same sizes, symmetric -> non-symmetric) is
    noticed by the pattern hash, and the call is repeated with a fresh analysis."""
    import torch

    S = synth.random_sparse_spd(1000, 3, 3, 1.0, "f64")
    C = _row_permuted(S, np.random.default_rng(12).permutation(S.d))  # same sizes, non-symmetric pattern
    shift = 20.0
    D = dev(S, shift=shift)
    a, b = oracle_lib.gershgorin(S, shift)
    say("grad pattern cache: first and second call")
    r1, g1 = ld.ld_logdet_cheb_grad(D, a, b, 11, 8, 4)
    r2, g2 = ld.ld_logdet_cheb_grad(D, a, b, 11, 8, 4)
    assert r1["logdet"] == r2["logdet"] and r1["grad_shift"] == r2["grad_shift"] and torch.equal(g1, g2)
    o = oracle_lib.logdet_grad(S, a, b, 11, 8, seed=4, shift=shift)
    assert entrywise(g1.cpu().numpy(), o["grad"]) <= 1e-10
    # the same device arrays now hold C's pattern and values
    D.row_ptr.copy_(torch.tensor(C.row_ptr, device=D.row_ptr.device))
    D.col.copy_(torch.tensor(C.col, device=D.col.device))
    D.values.copy_(torch.tensor(C.val, device=D.values.device))
    a2, b2 = oracle_lib.gershgorin(C, shift)
    assert a2 > 0
    say("grad pattern cache: pattern rewritten in place")
    r3, g3 = ld.ld_logdet_cheb_grad(D, a2, b2, 11, 8, 4)
    o3 = oracle_lib.logdet_grad(C, a2, b2, 11, 8, seed=4, shift=shift)
    assert entrywise(g3.cpu().numpy(), o3["grad"]) <= 1e-10
    assert rel(r3["logdet"], o3["gamma"]) <= 1e-10


def _row_permuted(B, perm):
    """P B: row i of the result is row perm[i] of B (columns and values kept, still sorted)."""
    lens = np.diff(B.row_ptr)[perm]
    rp = np.zeros(B.d + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    idx = np.concatenate([np.arange(B.row_ptr[r], B.row_ptr[r + 1]) for r in perm])
    return synth.CSR(B.d, rp, B.col[idx].copy(), B.val[idx].copy(), B.storage)


def test_torch_sparse_csr_front_end(ld, oracle_lib):
    """logdet() on a torch sparse CSR tensor: the value matches the oracle, and backward through
    the tensor's values matches the library's gradient entry point."""
    import torch

    B = synth.random_sparse_spd(3000, 3, 21, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B)
    crow = torch.tensor(B.row_ptr, device="cuda")
    col = torch.tensor(B.col.astype(np.int64), device="cuda")
    vals = torch.tensor(B.val, device="cuda", requires_grad=True)
    with warnings.catch_warnings():  # torch marks sparse CSR support as beta
        warnings.simplefilter("ignore", UserWarning)
        T = torch.sparse_csr_tensor(crow, col, vals, size=(B.d, B.d))
    say("torch sparse CSR front end")
    est, se = ld.logdet(T, 20, 16, seed=6)
    o = oracle_lib.logdet(B, a, b, 20, 16, seed=6)
    assert est.dtype == torch.float64 and rel(float(est.detach()), o["gamma"], floor_for(a, b, 20, B.d, 1e-10)) <= 1e-10
    assert rel(se, o["std_err"]) <= 1e-8
    est.backward()
    r, g = ld.ld_logdet_cheb_grad(dev(B), a, b, 20, 16, 6)
    assert torch.allclose(vals.grad, g.to(vals.grad.dtype), rtol=0, atol=1e-12 * float(g.abs().max()))
    est2, se2 = ld.logdet(T.detach(), 20, 16, seed=6)
    assert float(est2) == float(est.detach()) and se2 == se


@pytest.mark.parametrize("stride", [0, 3])
def test_grad_bitwise_reproducible(ld, stride):
    """No atomics on the gradient path: each stored entry is accumulated by the row that owns it
    and every reduction runs in a fixed order, so repeated calls agree bit for bit."""
    import torch

    B = synth.random_sparse_spd(20000, 5, 41, 1.0, "f32")
    D = dev(B, shift=0.05)
    say(f"grad reproducible stride={stride}")
    a, b = ld.ld_gershgorin(D)
    r1, g1 = ld.ld_logdet_cheb_grad(D, a, b, 24, 32, 13, ckpt_stride=stride)
    r2, g2 = ld.ld_logdet_cheb_grad(D, a, b, 24, 32, 13, ckpt_stride=stride)
    assert r1["logdet"] == r2["logdet"] and r1["grad_shift"] == r2["grad_shift"]
    assert torch.equal(g1, g2)


def test_grad_full_store_planned_per_form(ld):
    """A caller workspace too small for the plain form's full checkpoint store but large enough for
    the paired form's: a symmetric pattern runs the paired form and keeps every W_k (no
    recomputation), and the result equals the default call's bit for bit."""
    import torch

    B = synth.random_sparse_spd(20000, 5, 41, 1.0, "f32")
    D = dev(B, shift=0.05)
    a, b = ld.ld_gershgorin(D)
    n, M = 50, 32
    full = ld.ld_workspace_bytes(D, n, M, 2)  # either form with every W_k kept
    ws = torch.empty(int(full * 0.7) // 256 * 256, dtype=torch.uint8, device="cuda")
    say("grad full store planned per form")
    r1, g1 = ld.ld_logdet_cheb_grad(D, a, b, n, M, 13, workspace=ws, timing=True)
    assert r1["kernel_launches"] == (n + 1) // 2
    r2, g2 = ld.ld_logdet_cheb_grad(D, a, b, n, M, 13)
    assert r1["logdet"] == r2["logdet"] and torch.equal(g1, g2)


@pytest.mark.parametrize("tile", [32, 96, 512])
def test_grad_caller_tile_height(ld, oracle_lib, tile):
    """The caller's tile height (opt->tile) also shapes the gradient's kernels, including tiles
    too tall for the LDS slice (read from global memory)."""
    B = synth.random_sparse_spd(3000, 4, 29, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B)
    say(f"grad tile={tile}")
    r, g = ld.ld_logdet_cheb_grad(dev(B, shift=0.1), a + 0.1, b + 0.1, 17, 8, 6, tile=tile)
    o = oracle_lib.logdet_grad(B, a + 0.1, b + 0.1, 17, 8, seed=6, shift=0.1)
    assert entrywise(g.cpu().numpy(), o["grad"]) <= 1e-10
    assert rel(r["grad_shift"], o["grad_shift"]) <= 1e-10
    assert rel(r["logdet"], o["gamma"]) <= 1e-10

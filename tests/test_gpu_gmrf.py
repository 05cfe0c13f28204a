"""GPU side of the GMRF maximum-likelihood experiment (Section 5.2): the FP64 quadratic form, the
log-likelihood curve against the oracle on the same probes, its derivative through the adjoint,
and the maximum-likelihood fit against the closed-form optimum."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests._gpu import U32, dev, floor_for, rel, say

pytestmark = pytest.mark.gpu

N = 128
RHO0 = -0.22


@pytest.fixture(scope="module")
def ld():
    import torch

    assert torch.cuda.is_available()
    import paper_1503_06394_amd as pkg

    pkg.lib()
    return pkg


@pytest.fixture(scope="module")
def field(ld):
    import torch

    from paper_1503_06394_amd.gmrf import GMRF

    L = synth.grid_laplacian_2d(N, "f64")
    D = dev(L)
    x = synth.gmrf_sample(N, RHO0, seed=5)
    return GMRF(D.row_ptr, D.col), torch.tensor(x, dtype=torch.float64, device="cuda"), x, L


def _xax(L, x):
    rows = L.row_of_entry()
    off = L.col != rows
    return float(np.sum(x[rows[off]] * x[L.col[off].astype(np.int64)]))


def _exact_loglik(rho, x, xax):
    t = np.pi * np.arange(1, N + 1) / (N + 1)
    lam = 2.0 * np.cos(t)[:, None] + 2.0 * np.cos(t)[None, :]
    return 0.5 * float(np.log(1.0 - rho * lam).sum()) - 0.5 * (float(x @ x) - rho * xax)


@pytest.mark.parametrize("shift", [0.0, 0.3])
def test_quadratic_form(ld, shift):
    import torch

    B = synth.random_sparse_spd(20_000, 4, 6, 1.0, "f32")
    x = np.random.default_rng(1).standard_normal(B.d)
    say(f"quadratic form d={B.d} shift={shift}")
    q = ld.ld_quadratic_form(dev(B, shift=shift), torch.tensor(x, device="cuda"))
    rows = B.row_of_entry()
    want = float(np.sum(x[rows] * B.val * x[B.col.astype(np.int64)])) + shift * float(x @ x)
    assert rel(q, want) < 1e-12


@pytest.mark.parametrize("method", [1, 2])
def test_loglik_curve_parity(ld, oracle_lib, field, method):
    g, xt, x, L = field
    n, M, seed = 40, 32, 9
    rhos = [-0.24, -0.22, -0.2, 0.1] if method == 1 else [-0.22]
    for rho in rhos:
        say(f"gmrf loglik N={N} rho={rho} method={method}")
        r = g.loglik(rho, xt, n, M, seed, method=method)
        J = synth.gmrf_grid_precision(N, rho, "f32")
        a, b = 1 - 4 * abs(rho), 1 + 4 * abs(rho)
        if method == 1:
            o = oracle_lib.logdet(J, a, b, n, M, seed=seed)
        else:
            o = oracle_lib.logabsdet(J, a, b, n, M, seed=seed)
        assert rel(r["logdet"], o["gamma"], floor_for(a, b, n, J.d, 1e-4, U32) if method == 1 else floor_for(a * a, b * b, n, J.d, 1e-4, U32)) <= 1e-4, rho
        rows = J.row_of_entry()
        q = float(np.sum(x[rows] * J.val * x[J.col.astype(np.int64)]))
        assert rel(r["quad"], q) < 1e-12, rho


def test_loglik_derivative(ld, oracle_lib, field):
    """dl/drho from the adjoint against central differences of the oracle's estimate (same
    probes, FP64 model) plus the closed-form derivative of the quadratic term."""
    g, xt, x, L = field
    n, M, seed, rho, h = 40, 32, 9, -0.2, 1e-4
    say("gmrf loglik derivative")
    ll, dll = g.loglik_grad(rho, xt, n, M, seed)

    def og(r):
        return oracle_lib.logdet(synth.gmrf_grid_precision(N, r, "f64"), 1 - 4 * abs(rho), 1 + 4 * abs(rho), n, M,
                                 seed=seed)["gamma"]

    dgamma = (og(rho + h) - og(rho - h)) / (2 * h)
    want = 0.5 * dgamma + 0.5 * _xax(L, x)
    assert rel(dll, want) < 1e-4, (dll, want)


def test_fit_recovers_ml_rho(ld, field):
    """The secant iteration on dl/drho lands on the stationary point of the estimated curve,
    which is within 2e-3 of the exact maximum-likelihood rho (closed-form spectrum) and within
    0.01 of the hidden rho = -0.22."""
    g, xt, x, L = field
    say("gmrf fit")
    f = g.fit(xt, -0.1, 40, 32, 9)
    xax = _xax(L, x)
    rs = np.linspace(-0.249, -0.15, 2000)
    exact = rs[int(np.argmax([_exact_loglik(r, x, xax) for r in rs]))]
    assert abs(f["dloglik"]) < 1e-3 * g.d
    assert abs(f["rho"] - exact) < 2e-3, (f["rho"], exact)
    assert abs(f["rho"] - RHO0) < 0.01

"""Pins of the grid-GMRF inputs of the maximum-likelihood experiment (Section 5.2): the precision
matrix, the exact sampler, and the premise that the likelihood peaks at the hidden rho; plus the
oracle's log det along the curve against the closed-form spectrum."""
from __future__ import annotations

import numpy as np
import pytest

import synth


def _exact_logdet(N, rho):
    t = np.pi * np.arange(1, N + 1) / (N + 1)
    lam = 2.0 * np.cos(t)[:, None] + 2.0 * np.cos(t)[None, :]
    return float(np.log(1.0 - rho * lam).sum())


def test_precision_is_identity_minus_rho_adjacency():
    N, rho = 7, -0.22
    J = synth.dense(synth.gmrf_grid_precision(N, rho, "f64"))
    L = synth.dense(synth.grid_laplacian_2d(N, "f64"))
    A = 4.0 * np.eye(N * N) - L
    assert np.array_equal(J, np.eye(N * N) - rho * A)


@pytest.mark.parametrize("rho", [-0.22, 0.0, 0.15])
def test_sampler_covariance_is_inverse_precision(rho):
    """x = S D^{-1/2} S z, so stacking the draws for z = e_1..e_d gives X with X X^T = J^{-1}."""
    N = 6
    X = synth.gmrf_sample(N, rho, z=np.eye(N * N))
    J = synth.dense(synth.gmrf_grid_precision(N, rho, "f64"))
    assert np.abs(X @ X.T - np.linalg.inv(J)).max() < 1e-12


def test_closed_form_spectrum_matches_dense():
    N, rho = 9, 0.2
    J = synth.dense(synth.gmrf_grid_precision(N, rho, "f64"))
    assert abs(np.linalg.slogdet(J)[1] - _exact_logdet(N, rho)) < 1e-12


def test_exact_likelihood_peaks_near_hidden_rho():
    """The experiment's premise: for one draw at rho = -0.22 on a 64 x 64 grid the exact
    log-likelihood (1/2) log det J - (1/2) x^T J x is maximised within 0.015 of -0.22."""
    N, rho0 = 64, -0.22
    x = synth.gmrf_sample(N, rho0, seed=3)
    L = synth.dense(synth.grid_laplacian_2d(N, "f64"))
    xAx = x @ ((4.0 * np.eye(N * N) - L) @ x)
    rhos = np.linspace(-0.249, 0.0, 250)
    ll = [0.5 * _exact_logdet(N, r) - 0.5 * (x @ x - r * xAx) for r in rhos]
    assert abs(rhos[int(np.argmax(ll))] - rho0) < 0.015


def test_oracle_logdet_along_the_curve(oracle_lib):
    """The oracle's Algorithm 1 estimate of log det J(rho) at the Gershgorin bounds is within five
    standard errors of the closed-form value along the curve."""
    N = 24
    for rho in (-0.24, -0.22, -0.1, 0.1):
        J = synth.gmrf_grid_precision(N, rho, "f64")
        a, b = 1 - 4 * abs(rho), 1 + 4 * abs(rho)
        r = oracle_lib.logdet(J, a, b, 60, 64, seed=4)
        assert abs(r["gamma"] - _exact_logdet(N, rho)) < 5 * r["std_err"] + 1e-9


def test_fit_root_finder_on_closed_form_derivative():
    """The maximum-likelihood search (bracketing, then Illinois regula falsi) driven by the exact
    derivative of the 128 x 128 grid's log-likelihood lands on the exact optimum, from either
    side and from far away (host logic only: the library is not called)."""
    import torch

    from paper_1503_06394_amd.gmrf import GMRF

    N = 128
    x = synth.gmrf_sample(N, -0.22, seed=5)
    L = synth.grid_laplacian_2d(N, "f64")
    t = np.pi * np.arange(1, N + 1) / (N + 1)
    lam = (2.0 * np.cos(t)[:, None] + 2.0 * np.cos(t)[None, :]).ravel()
    rows = L.row_of_entry()
    off = L.col != rows
    xax = float(np.sum(x[rows[off]] * x[L.col[off].astype(np.int64)]))

    class Exact(GMRF):
        def loglik_grad(self, rho, x, n, M, seed):
            return 0.0, -0.5 * float(np.sum(lam / (1.0 - rho * lam))) + 0.5 * xax

    g = Exact(torch.as_tensor(L.row_ptr), torch.as_tensor(L.col))
    rs = np.linspace(-0.2495, -0.15, 20000)
    dl = -0.5 * np.sum(lam[None, :] / (1.0 - rs[:, None] * lam[None, :]), axis=1) + 0.5 * xax
    exact = rs[int(np.argmin(np.abs(dl)))]
    for rho0 in (-0.1, 0.2, -0.24, -0.2):
        f = g.fit(None, rho0, 0, 1, 0)
        assert abs(f["rho"] - exact) < 1e-4, (rho0, f["rho"], exact)
        assert len(f["path"]) < 30

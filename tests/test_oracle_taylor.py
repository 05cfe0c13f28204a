"""Pins of the oracle's Taylor-series comparator (the accuracy comparison of Section 5.1).

Expected values come from the exact log det (numpy), powers of the eigenvalues, brute force
over all probe sign patterns, and the closed-form spectrum of the Dirichlet grid.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

import synth


def test_taylor_degree_zero_is_the_lift(oracle_lib):
    B = synth.random_sparse_spd(50, 3, 4, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B)
    r = oracle_lib.logdet_taylor(B, a, b, 0, 3, seed=2)
    assert r["gamma"] == 50 * math.log(a + b)


@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_taylor_degree_increment_diagonal(oracle_lib, n):
    """For a diagonal B every probe gives v^T A^k v = sum_i (1 - b_ii/(a+b))^k, so raising the
    degree from n-1 to n changes the estimate by -(1/n) sum_i x_i^n."""
    lam = np.array([0.3, 0.9, 1.7, 2.2, 3.1])
    a, b = 0.3, 3.1
    B = synth.diagonal_matrix(lam)
    x = 1.0 - lam / (a + b)
    g1 = oracle_lib.logdet_taylor(B, a, b, n, 2, seed=5)["gamma"]
    g0 = oracle_lib.logdet_taylor(B, a, b, n - 1, 2, seed=5)["gamma"]
    assert abs((g1 - g0) - (-np.sum(x ** n) / n)) < 1e-14


def test_taylor_converges_to_logdet(oracle_lib):
    """At high degree the series reaches log det: diagonal exactly, and a dense 10 x 10 SPD matrix
    through the mean over all 2^10 probe sign patterns (the exact trace)."""
    lam = np.array([0.5, 1.0, 2.0, 3.5])
    r = oracle_lib.logdet_taylor(synth.diagonal_matrix(lam), 0.5, 3.5, 2000, 1, seed=1)
    assert abs(r["gamma"] - np.log(lam).sum()) < 1e-12
    B = synth.random_sparse_spd(10, 3, 12, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B)
    V = np.array(list(itertools.product([1.0, -1.0], repeat=10)))
    r = oracle_lib.logdet_taylor(B, a, b, 600, V.shape[0], V=V)
    exact = np.linalg.slogdet(synth.dense(B))[1]
    assert abs(r["gamma"] - exact) < 1e-10 * abs(exact) + 1e-10


def test_taylor_shift_equals_stored_diagonal(oracle_lib):
    B = synth.random_sparse_spd(80, 3, 6, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B, 0.25)
    r1 = oracle_lib.logdet_taylor(B, a, b, 12, 4, seed=3, shift=0.25)
    diag = B.col == B.row_of_entry()
    B2 = synth.CSR(B.d, B.row_ptr, B.col, np.where(diag, B.val + 0.25, B.val), "f64", {})
    r2 = oracle_lib.logdet_taylor(B2, a, b, 12, 4, seed=3)
    assert abs(r1["gamma"] - r2["gamma"]) < 1e-12 * abs(r2["gamma"])


@pytest.mark.parametrize("n", [10, 20, 30, 50])
def test_chebyshev_more_accurate_than_taylor(oracle_lib, n):
    """Section 5.1's comparison, free of probe noise: on a diagonal matrix holding the spectrum of
    the 32 x 32 Dirichlet grid + 0.1 I (closed form), both estimators are exact polynomial traces,
    and at equal degree the Chebyshev interpolant is closer to log det than the Taylor series."""
    N = 32
    t = np.pi * np.arange(1, N + 1) / (N + 1)
    lam = (4.0 - 2.0 * np.cos(t)[:, None] - 2.0 * np.cos(t)[None, :]).ravel() + 0.1
    B = synth.diagonal_matrix(lam)
    exact = np.log(lam).sum()
    ch = oracle_lib.logdet(B, 0.1, 8.1, n, 1, seed=9)["gamma"]
    ta = oracle_lib.logdet_taylor(B, 0.1, 8.1, n, 1, seed=9)["gamma"]
    assert abs(ch - exact) < abs(ta - exact)
    assert abs(ch - exact) < 0.2 * abs(ta - exact)

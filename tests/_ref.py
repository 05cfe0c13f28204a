"""Independent reference computations used to pin the oracle and the GPU path.

Everything here is built from closed forms or numpy/scipy library routines (dense
eigendecompositions, numpy's Chebyshev interpolation at first-kind points), never from
the oracle's code, so that a mistake in the oracle shows up as a disagreement.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import chebyshev as npcheb


def grid2d_eigs(N: int) -> np.ndarray:
    """Eigenvalues of the N x N Dirichlet 5-point Laplacian."""
    t = 2.0 * np.cos(np.arange(1, N + 1) * math.pi / (N + 1))
    return (4.0 - t[:, None] - t[None, :]).ravel()


def grid3d_eigs(N: int) -> np.ndarray:
    """Eigenvalues of the N x N x N Dirichlet 7-point Laplacian."""
    t = 2.0 * np.cos(np.arange(1, N + 1) * math.pi / (N + 1))
    return (6.0 - t[:, None, None] - t[None, :, None] - t[None, None, :]).ravel()


def grid_eigvecs_1d(N: int) -> np.ndarray:
    """Orthonormal sine eigenvectors of the 1-D Dirichlet Laplacian, column p is mode p+1."""
    i = np.arange(1, N + 1)[:, None]
    p = np.arange(1, N + 1)[None, :]
    return math.sqrt(2.0 / (N + 1)) * np.sin(i * p * math.pi / (N + 1))


def log_interval_fn(a: float, b: float):
    """f(x) = log(((b - a) x + (a + b)) / 2): log on [a, b] pulled back to [-1, 1]."""
    return lambda x: np.log(((b - a) * np.asarray(x) + (a + b)) / 2.0)


def cheb_coeffs(a: float, b: float, n: int) -> np.ndarray:
    """Degree-n interpolant of log on [a, b] at first-kind Chebyshev points (numpy routine)."""
    return npcheb.chebinterpolate(log_interval_fn(a, b), n)


def p_n_on_interval(a: float, b: float, n: int, lam: np.ndarray) -> np.ndarray:
    """p_n(lambda) for lambda in original units (interpolant of log on [a, b])."""
    x = (2.0 * np.asarray(lam) - (a + b)) / (b - a)
    return npcheb.chebval(x, cheb_coeffs(a, b, n))


def dp_n_on_interval(a: float, b: float, n: int, lam: np.ndarray) -> np.ndarray:
    """d/d lambda of p_n(lambda) (chain rule through the affine map)."""
    x = (2.0 * np.asarray(lam) - (a + b)) / (b - a)
    return npcheb.chebval(x, npcheb.chebder(cheb_coeffs(a, b, n))) * 2.0 / (b - a)


def pn_matrix(Bd: np.ndarray, a: float, b: float, n: int, deriv: bool = False) -> np.ndarray:
    """p_n(B) (or p_n'(B)) of a dense symmetric matrix via its eigendecomposition."""
    lam, Q = np.linalg.eigh(Bd)
    vals = dp_n_on_interval(a, b, n, lam) if deriv else p_n_on_interval(a, b, n, lam)
    return (Q * vals) @ Q.T


def brute_probe_values(Bd: np.ndarray, a: float, b: float, n: int, V: np.ndarray) -> np.ndarray:
    """Exact per-probe values v_j^T p_n(B) v_j for a dense symmetric B (V is m x d)."""
    P = pn_matrix(Bd, a, b, n)
    return np.einsum("jd,de,je->j", V, P, V)


def all_sign_vectors(d: int) -> np.ndarray:
    """All 2^d Rademacher vectors, shape (2^d, d)."""
    k = np.arange(2 ** d)[:, None]
    bits = (k >> np.arange(d)[None, :]) & 1
    return 1.0 - 2.0 * bits


def splitmix64_published(path: str) -> list:
    with open(path) as fh:
        return [int(x) for x in fh.read().split("\n") if x.strip() and not x.startswith("#")]


def single_probe_variance_grid2d(N: int, a: float, b: float, n: int, shift: float) -> tuple:
    """Exact mean and single-probe variance of v^T p_n(L + shift I) v for the 2-D grid.

    Mean = sum p(lambda); variance = 2 (||P||_F^2 - sum_i P_ii^2) with P = p_n(L + shift I).
    The diagonal of P comes from the separable sine eigenvectors.
    """
    U = grid_eigvecs_1d(N)
    t = 2.0 * np.cos(np.arange(1, N + 1) * math.pi / (N + 1))
    lam = 4.0 - t[:, None] - t[None, :] + shift  # (p, q)
    P = p_n_on_interval(a, b, n, lam)
    mean = float(P.sum())
    fro2 = float((P ** 2).sum())
    U2 = U ** 2  # (i, p)
    diag = U2 @ P @ U2.T  # (i, j): P_{(i,j),(i,j)}
    var = 2.0 * (fro2 - float((diag ** 2).sum()))
    return mean, var

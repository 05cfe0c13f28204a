"""Pins of the oracle's Lanczos spectral estimate (the step before the path: bounds on the
extreme eigenvalues or singular values, Section 3.2).  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth


def _krylov_ritz(A: np.ndarray, v: np.ndarray, k: int) -> np.ndarray:
    """Rayleigh-Ritz values of A on span{v, Av, ..., A^(k-1) v}, from a QR factorisation of that
    power basis: the textbook characterisation, independent of the three-term recurrence."""
    K = np.empty((A.shape[0], k))
    x = v.copy()
    for i in range(k):
        K[:, i] = x / np.linalg.norm(x)
        x = A @ K[:, i]
    Q, _ = np.linalg.qr(K)
    return np.linalg.eigvalsh(Q.T @ A @ Q)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("gram", [False, True])
def test_lanczos_is_rayleigh_ritz_on_the_krylov_space(k, gram):
    if gram:
        B = synth.random_nonsingular(70, 4, 3, 3.0, "f64")
        Dn = synth.dense(B)
        A = Dn.T @ Dn
        shift = 0.0
    else:
        B = synth.random_sparse_spd(70, 3, 8, 1.0, "f64")
        shift = 0.35
        A = synth.dense(B) + shift * np.eye(B.d)
    v = oracle.probe(11, 0, B.d)
    rr = _krylov_ritz(A, v, k)
    lo, hi, al, be = oracle.lanczos_extremes(B, k, seed=11, shift=shift, gram=gram)
    scale = np.abs(rr).max()
    assert abs(lo - rr[0]) <= 1e-11 * scale and abs(hi - rr[-1]) <= 1e-11 * scale
    assert al.shape == (k,) and be.shape == (k - 1,)


def test_lanczos_full_space_reaches_the_spectrum_ends():
    B = synth.random_sparse_spd(40, 3, 2, 1.0, "f64")
    ev = np.linalg.eigvalsh(synth.dense(B))
    lo, hi, _, _ = oracle.lanczos_extremes(B, 40, seed=5)
    assert abs(lo - ev[0]) <= 1e-10 * ev[-1] and abs(hi - ev[-1]) <= 1e-10 * ev[-1]


def test_lanczos_ritz_values_interlace_and_converge():
    """Ritz values stay inside [lambda_min, lambda_max] and move outwards as the space grows;
    on the 32 x 32 grid (closed-form spectrum) both ends converge."""
    B = synth.grid_laplacian_2d(32, "f64")
    p = np.arange(1, 33) * np.pi / 33
    lam = (4 - 2 * np.cos(p)[:, None] - 2 * np.cos(p)[None, :]).ravel() + 0.1
    prev_lo, prev_hi = np.inf, -np.inf
    for k in (2, 5, 10, 20, 40, 80):
        lo, hi, _, _ = oracle.lanczos_extremes(B, k, seed=1, shift=0.1)
        assert lam.min() * (1 - 1e-12) <= lo <= prev_lo * (1 + 1e-12)
        assert prev_hi * (1 - 1e-12) <= hi <= lam.max() * (1 + 1e-12)
        prev_lo, prev_hi = lo, hi
    lo, hi, _, _ = oracle.lanczos_extremes(B, 300, seed=1, shift=0.1)
    assert lo <= lam.min() * 1.02 and hi >= lam.max() * (1 - 2e-3)


def test_lanczos_shift_moves_every_ritz_value():
    B = synth.random_sparse_spd(90, 3, 4, 1.0, "f64")
    lo0, hi0, al0, be0 = oracle.lanczos_extremes(B, 12, seed=2)
    lo1, hi1, al1, be1 = oracle.lanczos_extremes(B, 12, seed=2, shift=2.5)
    assert np.allclose(al1, al0 + 2.5, rtol=0, atol=1e-12) and np.allclose(be1, be0, rtol=0, atol=1e-12)
    assert abs(lo1 - lo0 - 2.5) <= 1e-12 * hi1 and abs(hi1 - hi0 - 2.5) <= 1e-12 * hi1

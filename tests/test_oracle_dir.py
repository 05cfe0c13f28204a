"""Pins of the oracle's forward-mode directional derivative (ldo_logdet_dir), the check the
full-size gradient parity uses where the oracle's reverse mode cannot store its vectors.

The estimate is a polynomial in the entries of B (a and b fixed), so central differences of the
oracle's own estimate are exact up to O(h^2); the reverse mode (ldo_logdet_grad) is a different
algorithm whose contraction with the direction must agree to rounding."""
from __future__ import annotations

import numpy as np
import pytest

import synth


def _direction(B, seed: int):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, B.nnz), float(rng.uniform(-1.0, 1.0))


def _perturbed(B, e, h):
    return synth.CSR(B.d, B.row_ptr, B.col, B.val + h * e, "f64")


@pytest.mark.parametrize("kind", ["spd", "nonsymmetric", "grid"])
def test_directional_derivative_vs_central_differences(oracle_lib, kind):
    if kind == "spd":
        B, shift = synth.random_sparse_spd(60, 3, 8, 1.0, "f64"), 0.2
    elif kind == "nonsymmetric":
        B, shift = synth.lower_triangular_nonsymmetric(50, 3, 5), 0.0
    else:
        B, shift = synth.grid_laplacian_2d(9, "f64"), 0.3
    a, b = oracle_lib.gershgorin(B, shift)
    a, b = 0.9 * a, 1.1 * b
    n, m, seed = 17, 6, 4
    e, es = _direction(B, 11)
    dg = oracle_lib.logdet_dir(B, a, b, n, m, e, es, seed=seed, shift=shift)
    h = 1e-5
    gp = oracle_lib.logdet(_perturbed(B, e, h), a, b, n, m, seed=seed, shift=shift + h * es)["gamma"]
    gm = oracle_lib.logdet(_perturbed(B, e, -h), a, b, n, m, seed=seed, shift=shift - h * es)["gamma"]
    fd = (gp - gm) / (2 * h)
    assert abs(dg - fd) <= 1e-6 * max(abs(fd), 1.0), (dg, fd)


@pytest.mark.parametrize("kind", ["spd", "nonsymmetric"])
def test_directional_derivative_matches_reverse_mode(oracle_lib, kind):
    if kind == "spd":
        B, shift = synth.random_sparse_spd(200, 4, 21, 1.0, "f64"), 0.1
    else:
        B, shift = synth.lower_triangular_nonsymmetric(150, 3, 7), 0.0
    a, b = oracle_lib.gershgorin(B, shift)
    a, b = 0.95 * a, 1.05 * b
    n, m, seed = 23, 5, 9
    e, es = _direction(B, 3)
    dg = oracle_lib.logdet_dir(B, a, b, n, m, e, es, seed=seed, shift=shift)
    r = oracle_lib.logdet_grad(B, a, b, n, m, seed=seed, shift=shift)
    rev = float(np.dot(r["grad"], e) + r["grad_shift"] * es)
    assert abs(dg - rev) <= 1e-11 * max(abs(rev), 1.0), (dg, rev)


def test_directional_derivative_degree_zero_and_one(oracle_lib):
    """n = 0: the estimate d log((a+b)/2) does not move.  n = 1, in the [a, b] form: Gamma = c_0 d +
    c_1 v^T At v with At = (2 B' - (a+b) I)/(b - a), B' = B + shift I, so the derivative along E' =
    E + e_shift I is c_1 v^T (2 E'/(b - a)) v, c_1 the degree-1 coefficient of log on [a, b]."""
    B = synth.random_sparse_spd(40, 2, 5, 1.0, "f64")
    a, b = oracle_lib.gershgorin(B)
    e, es = _direction(B, 2)
    assert oracle_lib.logdet_dir(B, a, b, 0, 3, e, es, seed=1) == 0.0
    # c_1 of eq. (1) for log on [a, b] at degree 1: (2/2) sum_k f(x_k) x_k over the nodes +-1/sqrt(2)
    x = np.array([np.cos(np.pi / 4), np.cos(3 * np.pi / 4)])
    f = np.log(((b - a) * x + (a + b)) / 2.0)
    c1 = float(np.sum(f * x))
    dense_e = np.zeros((B.d, B.d))
    rows = np.repeat(np.arange(B.d), np.diff(B.row_ptr))
    dense_e[rows, B.col] = e
    dense_e += es * np.eye(B.d)
    import oracle

    want = 0.0
    for j in range(3):
        v = oracle.probe(1, j, B.d)
        want += c1 * (2.0 / (b - a)) * float(v @ dense_e @ v) / 3
    got = oracle_lib.logdet_dir(B, a, b, 1, 3, e, es, seed=1)
    assert abs(got - want) <= 1e-12 * max(abs(want), 1.0), (got, want)

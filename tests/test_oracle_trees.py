"""Pins of the oracle's spanning-tree counting (Section 3.3) against closed forms.

Expected values come from textbook counts (wheels: Lucas numbers, complete graphs: Cayley's
formula), from a dense Laplacian built here with numpy, and from the exact trace over all
probe sign patterns; none re-types the oracle's construction.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

import synth


def _dense_adj(G) -> np.ndarray:
    A = np.zeros((G.d, G.d))
    A[np.repeat(np.arange(G.d), np.diff(G.row_ptr)), G.col.astype(np.int64)] = 1.0
    return A


def _dense(L) -> np.ndarray:
    M = np.zeros((L.d, L.d))
    M[np.repeat(np.arange(L.d), np.diff(L.row_ptr)), L.col.astype(np.int64)] = L.val
    return M


def _lucas(k: int) -> int:
    a, b = 2, 1
    for _ in range(k):
        a, b = b, a + b
    return a


@pytest.mark.parametrize("k,count", [(3, 16), (4, 45), (5, 121), (10, 15125), (20, 228826125)])
def test_wheel_minor_counts_trees(oracle_lib, k, count):
    """Wheel W_k has L_2k - 2 spanning trees (L: Lucas numbers); the listed counts are that."""
    assert _lucas(2 * k) - 2 == count
    L, dmax = oracle_lib.laplacian_minor(synth.wheel_graph(k), 0)
    assert dmax == 3
    sign, logdet = np.linalg.slogdet(_dense(L))
    assert sign == 1.0 and abs(logdet - math.log(count)) < 1e-12 * math.log(count)


@pytest.mark.parametrize("nv", [3, 4, 5, 6, 8])
def test_complete_graph_minor_cayley(oracle_lib, nv):
    """K_n has n^(n-2) spanning trees (Cayley); any vertex of K_n is a hub."""
    hub = nv // 2
    L, dmax = oracle_lib.laplacian_minor(synth.complete_graph(nv), hub)
    assert dmax == nv - 1
    sign, logdet = np.linalg.slogdet(_dense(L))
    assert sign == 1.0 and abs(logdet - (nv - 2) * math.log(nv)) < 1e-12 * max(1.0, (nv - 2) * math.log(nv))


@pytest.mark.parametrize("hub_at", ["first", "middle", "last"])
def test_minor_is_laplacian_without_hub_row(oracle_lib, hub_at):
    """L(hub) = (D - A) with the hub's row and column deleted, columns sorted, spectrum in
    [1, 2 Delta_max - 1] (Section 3.3)."""
    G = synth.hub_graph(60, 3, 5)
    nv = G.d
    hub = {"first": 0, "middle": nv // 2, "last": nv - 1}[hub_at]
    perm = np.arange(nv)
    perm[[0, hub]] = perm[[hub, 0]]  # move the generator's hub (vertex 0) to position `hub`
    u, v = np.nonzero(np.triu(_dense_adj(G)))
    Gp = synth.graph_from_edges(nv, perm[u], perm[v])
    A = _dense_adj(Gp)
    Lfull = np.diag(A.sum(axis=1)) - A
    keep = np.arange(nv) != hub
    want = Lfull[np.ix_(keep, keep)]
    L, dmax = oracle_lib.laplacian_minor(Gp, hub)
    assert np.array_equal(_dense(L), want)
    for r in range(L.d):
        assert np.all(np.diff(L.col[L.row_ptr[r]:L.row_ptr[r + 1]]) > 0)
    assert dmax == int(A.sum(axis=1)[keep].max())
    ev = np.linalg.eigvalsh(want)
    assert ev.min() >= 1.0 - 1e-12 and ev.max() <= 2 * dmax - 1 + 1e-12


@pytest.mark.parametrize("method,n", [(0, 30), (1, 60)])
def test_tree_estimate_exact_trace(oracle_lib, method, n):
    """Averaged over all 2^d probe sign patterns the estimate is the exact trace of the
    polynomial, which for these degrees equals log tau(W_10) = log 15125 within the Chebyshev
    interpolation error on [1, 5] (Algorithm 1) or [1, 25] (Algorithm 2 on L^2)."""
    G = synth.wheel_graph(10)
    d = 10
    V = np.array(list(itertools.product([1.0, -1.0], repeat=d)))
    r = oracle_lib.log_spanning_trees(G, 0, n, V.shape[0], V=V, method=method)
    assert abs(r["gamma"] - math.log(15125)) < 1e-8


def test_star_graph_has_one_tree(oracle_lib):
    """A star (hub plus leaves) has L(hub) = I and exactly one spanning tree."""
    nv = 7
    G = synth.graph_from_edges(nv, np.zeros(nv - 1, dtype=np.int64), np.arange(1, nv))
    r = oracle_lib.log_spanning_trees(G, 0, 10, 4, seed=1)
    assert r["gamma"] == 0.0 and r["delta_max"] == 1


def test_tree_estimate_statistical(oracle_lib):
    """A random hub graph (d = 400): the estimate is within 5 standard errors of the dense
    log det of L(hub)."""
    G = synth.hub_graph(400, 3, 9)
    r = oracle_lib.log_spanning_trees(G, 0, 40, 200, seed=11, method=1)
    L = r["minor"]
    exact = np.linalg.slogdet(_dense(L))[1]
    assert abs(r["gamma"] - exact) < 5 * r["std_err"] + 1e-6 * exact


def test_spanning_tree_corollary_guarantee(oracle_lib):
    """The spanning-tree corollary as an inequality: for the wheel W_20 (Delta_max = Delta_avg = 3),
    eps = 0.5 < 2/(Delta_avg - 1) and zeta = 0.2, Algorithm 2 with m and n at the corollary's
    requirement (Theorem 2's M and N at eps (Delta_avg - 1)/4 and kappa = 2 Delta_max - 1) lands within
    eps log tau of log tau in every one of 3 runs."""
    eps, zeta = 0.5, 0.2
    m_req, n_req = oracle_lib.thm2_params(eps * (3 - 1) / 4, 2 * 3 - 1, zeta)
    m, n = int(math.ceil(m_req)), int(math.ceil(n_req))
    log_tau = math.log(_lucas(40) - 2)
    for seed in range(3):
        r = oracle_lib.log_spanning_trees(synth.wheel_graph(20), 0, n, m, seed=seed, method=1)
        assert abs(r["gamma"] - log_tau) <= eps * log_tau


@pytest.mark.parametrize("method", [0, 1])
def test_tree_estimate_uses_the_corollary_interval(oracle_lib, method):
    """At low degree the estimate depends on the interval: averaged over all sign patterns it must
    equal the trace of the degree-3 first-kind Chebyshev interpolant of log on [1, 2 Delta_max - 1]
    (Algorithm 1 on L(hub)), or half that of log on [1, (2 Delta_max - 1)^2] over L(hub)^2
    (Algorithm 2), built here with numpy from the minor's eigenvalues."""
    from numpy.polynomial import chebyshev as C

    G = synth.wheel_graph(6)
    L, dmax = oracle_lib.laplacian_minor(G, 0)
    lam = np.linalg.eigvalsh(_dense(L))
    hi = 2.0 * dmax - 1.0
    if method == 0:
        a, b, x = 1.0, hi, lam
    else:
        a, b, x = 1.0, hi * hi, lam * lam
    coef = C.chebinterpolate(lambda t: np.log(((b - a) * t + (a + b)) / 2.0), 3)
    want = float(C.chebval((2.0 * x - (a + b)) / (b - a), coef).sum()) * (1.0 if method == 0 else 0.5)
    V = np.array(list(itertools.product([1.0, -1.0], repeat=L.d)))
    r = oracle_lib.log_spanning_trees(G, 0, 3, V.shape[0], V=V, method=method)
    assert abs(r["gamma"] - want) < 1e-11 * max(1.0, abs(want))

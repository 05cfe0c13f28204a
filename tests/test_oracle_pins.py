"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names the passage it pins.  None of them re-types the oracle's own formula:
expected values come from closed forms, numpy/scipy routines, brute force over all
probe sign patterns, or the published SplitMix64 sequence.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import synth
from tests import _ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------------------
# Chebyshev coefficients, Section 2.1 eq. (1)
# --------------------------------------------------------------------------------------

def _alg1_series_coeffs(delta: float, kmax: int) -> np.ndarray:
    """Chebyshev series of h(x) = log(1 - ((1-2 delta)x + 1)/2) on [-1, 1] in closed form.

    h(x) = log(((1-2d)(-x) + 1)/2) and log(((b-a)x + (a+b))/2) = 2 log((sqrt a + sqrt b)/2)
    + sum_k (2/k)(-1)^{k+1} r^k T_k(x), r = (sqrt b - sqrt a)/(sqrt b + sqrt a), from the
    generating function log(1 - 2tx + t^2) = -2 sum_k t^k T_k(x)/k; T_k(-x) = (-1)^k T_k(x).
    """
    a, b = delta, 1.0 - delta
    r = (math.sqrt(b) - math.sqrt(a)) / (math.sqrt(b) + math.sqrt(a))
    k = np.arange(kmax + 1, dtype=np.float64)
    coef = np.zeros(kmax + 1)
    coef[0] = 2.0 * math.log((math.sqrt(a) + math.sqrt(b)) / 2.0)
    kk = k[1:]
    coef[1:] = (2.0 / kk) * (-1.0) ** (kk + 1) * r ** kk * (-1.0) ** kk
    return coef


def _alias(series: np.ndarray, n: int) -> np.ndarray:
    """Interpolation at n+1 first-kind nodes folds T_{2l(n+1) +- j} onto (-1)^l T_j."""
    c = np.zeros(n + 1)
    P = 2 * (n + 1)
    for m, am in enumerate(series):
        l, rem = divmod(m, P)
        sign = (-1.0) ** l
        if rem <= n:
            c[rem] += sign * am
        elif rem == n + 1:
            continue  # T_{(2l+1)(n+1)} vanishes at every node
        else:
            c[P - rem] += -sign * am  # T_{P - j} = -T_j at the nodes
    return c


@pytest.mark.parametrize("a,b,n", [(0.1, 8.1, 30), (1.0, 23.0, 50), (0.09, 12.09, 60), (0.01, 8.01, 100),
                                   (0.3, 0.7, 0), (0.3, 0.7, 1), (2.0, 3.0, 7)])
def test_coeffs_closed_form_series_with_aliasing(oracle_lib, a, b, n):
    """eq. (1) coefficients equal the aliased closed-form Chebyshev series of the log."""
    delta = a / (a + b)
    c = oracle_lib.cheb_coeffs_alg1(delta, n)
    series = _alg1_series_coeffs(delta, 40 * (n + 1) + 4000)
    expect = _alias(series, n)
    np.testing.assert_allclose(c, expect, rtol=0, atol=1e-13)


def test_coeffs_closed_form_values_grid32(oracle_lib):
    """for [a, b] = [0.1, 8.1], n = 30 the B-form coefficients are c0 = 0.916290763512757,
    c1 = 1.599999934894294 (closed-form series); the A-form of Algorithm 1 has c_j^A = (-1)^j c_j^B
    with log(a+b) removed from c_0."""
    c = oracle_lib.cheb_coeffs_alg1(0.1 / 8.2, 30)
    assert abs((c[0] + math.log(8.2)) - 0.916290763512757) < 1e-13
    assert abs(-c[1] - 1.599999934894294) < 1e-13


@pytest.mark.parametrize("n", [0, 1, 2, 5, 17, 64])
def test_coeffs_match_numpy_first_kind_interpolation(oracle_lib, n):
    """eq. (1) is interpolation at first-kind nodes; numpy's chebinterpolate is the same object."""
    delta = 0.07
    h = lambda x: np.log(1.0 - ((1.0 - 2.0 * delta) * x + 1.0) / 2.0)
    np.testing.assert_allclose(oracle_lib.cheb_coeffs_alg1(delta, n), npcheb.chebinterpolate(h, n),
                               rtol=0, atol=2e-14)


@pytest.mark.parametrize("n", [0, 3, 10, 31])
def test_coeffs_reproduce_chebyshev_polynomials(oracle_lib, n):
    """f = T_i gives c = e_i (c_0 carries weight 1/(n+1), the others 2/(n+1)); p_n(x_k) = f(x_k)."""
    x = oracle_lib.cheb_nodes(n)
    np.testing.assert_allclose(x, np.cos(math.pi * (np.arange(n + 1) + 0.5) / (n + 1)), atol=0, rtol=1e-15)
    for i in range(n + 1):
        fx = np.cos(i * np.arccos(x))
        c = oracle_lib.cheb_coeffs_from_values(fx)
        e = np.zeros(n + 1)
        e[i] = 1.0
        np.testing.assert_allclose(c, e, atol=1e-13)
    f = np.exp(x) * np.sin(3 * x)
    c = oracle_lib.cheb_coeffs_from_values(f)
    np.testing.assert_allclose(npcheb.chebval(x, c), f, atol=1e-13)


# --------------------------------------------------------------------------------------
# Probes: Section 2.2 (Rademacher) with the SplitMix64 counter hash
# --------------------------------------------------------------------------------------

def test_probe_hash_matches_published_splitmix64(oracle_lib):
    """Probe word ctr is output ctr+1 of SplitMix64 from state `seed`; bits j&63 give probe j."""
    words = _ref.splitmix64_published(os.path.join(GOLDEN, "splitmix64_state1234567.txt"))
    seed = 1234567
    for ctr, w in enumerate(words):
        # row 0, probe block ctr -> ctr = (0 << 16) | (j >> 6)
        for bit in range(64):
            j = 64 * ctr + bit
            expect = -1 if (w >> bit) & 1 else 1
            assert oracle_lib.probe_sign(seed, j, 0) == expect


def test_probe_statistics(oracle_lib):
    """Rademacher: balanced signs, uncorrelated across probes and rows."""
    d = 20000
    V = np.stack([oracle_lib.probe(7, j, d) for j in range(8)])
    assert set(np.unique(V)) == {-1.0, 1.0}
    assert abs(V.mean()) < 4.0 / math.sqrt(V.size)
    G = V @ V.T / d
    off = G[~np.eye(8, dtype=bool)]
    assert np.abs(off).max() < 5.0 / math.sqrt(d)
    lag = (V[:, 1:] * V[:, :-1]).mean()
    assert abs(lag) < 5.0 / math.sqrt(V.size)
    # distinct seeds differ
    assert not np.array_equal(oracle_lib.probe(7, 0, 256), oracle_lib.probe(8, 0, 256))


# --------------------------------------------------------------------------------------
# Algorithm 1: exact special cases
# --------------------------------------------------------------------------------------

def test_degree_zero_closed_form(oracle_lib):
    """n = 0 gives Gamma = d log((a+b)/2) for any probes."""
    B = synth.grid_laplacian_2d(8)
    r = oracle_lib.logdet(B, 0.1, 8.1, 0, 5, seed=3, shift=0.1)
    assert abs(r["gamma"] - B.d * math.log(4.1)) <= 1e-13 * abs(r["gamma"])


def test_diagonal_matrix_exact_at_nodes(oracle_lib):
    """a diagonal B with entries at the mapped nodes gives Gamma = sum log b_ii exactly,
    because v_i^2 = 1 and the interpolant equals log at the nodes."""
    a, b, n = 0.5, 9.0, 12
    x = np.cos(math.pi * (np.arange(n + 1) + 0.5) / (n + 1))
    lam = ((b - a) * x + (a + b)) / 2.0
    diag = np.resize(lam, 40)
    B = synth.diagonal_matrix(diag)
    for seed in (0, 1, 99):
        r = oracle_lib.logdet(B, a, b, n, 3, seed=seed)
        assert abs(r["gamma"] - np.log(diag).sum()) <= 1e-13 * abs(np.log(diag).sum())


def test_diagonal_matrix_any_entries(oracle_lib):
    """for any diagonal B every probe gives sum_i p_n(b_ii)."""
    rng = np.random.default_rng(0)
    a, b, n = 0.2, 5.0, 23
    diag = rng.uniform(a, b, size=57)
    B = synth.diagonal_matrix(diag)
    r = oracle_lib.logdet(B, a, b, n, 4, seed=5)
    expect = _ref.p_n_on_interval(a, b, n, diag).sum()
    np.testing.assert_allclose(r["s"], expect, rtol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 9, 30])
def test_per_probe_brute_force(oracle_lib, n):
    """Each probe's value equals v^T p_n(B) v with p_n(B) from a dense eigendecomposition and
    numpy's first-kind interpolant of log on [a, b] (the mapped reading of Algorithm 1)."""
    B = synth.random_sparse_spd(60, k_off=3, mseed=11, storage="f64")
    a, b = oracle_lib.gershgorin(B)
    m = 6
    V = np.stack([oracle_lib.probe(42, j, B.d) for j in range(m)])
    r = oracle_lib.logdet(B, a, b, n, m, V=V)
    expect = _ref.brute_probe_values(synth.dense(B), a, b, n, V)
    np.testing.assert_allclose(r["s"], expect, rtol=1e-12)
    # the seeded path with the same seed produces the same probes
    r2 = oracle_lib.logdet(B, a, b, n, m, seed=42)
    np.testing.assert_allclose(r2["s"], r["s"], rtol=0, atol=0)


def test_nonsymmetric_probe_vector_rejected_shape(oracle_lib):
    B = synth.grid_laplacian_2d(4)
    with pytest.raises(ValueError):
        oracle_lib.logdet(B, 0.1, 8.1, 4, 2, V=np.ones((3, B.d)))


def test_enumeration_equals_trace(oracle_lib):
    """averaging over all 2^d sign vectors gives tr p_n(B) = sum_i p_n(lambda_i) exactly, and
    Lemma 7 bounds |log det B - tr p_n| (Section 4.1)."""
    B = synth.random_sparse_spd(11, k_off=2, mseed=5, storage="f64")
    Bd = synth.dense(B)
    a, b = oracle_lib.gershgorin(B)
    n = 8
    V = _ref.all_sign_vectors(B.d)
    r = oracle_lib.logdet(B, a, b, n, V.shape[0], V=V)
    lam = np.linalg.eigvalsh(Bd)
    tr = _ref.p_n_on_interval(a, b, n, lam).sum()
    assert abs(r["gamma"] - tr) <= 1e-12 * abs(tr)
    exact = np.log(lam).sum()
    delta = a / (a + b)
    assert abs(exact - (tr)) <= oracle_lib.lemma_bound(delta, n, B.d)


def test_scale_invariance(oracle_lib):
    """Gamma(sB; sa, sb) = Gamma(B; a, b) + d log s with the same probes (the mapped matrix
    is unchanged; only the log lift moves)."""
    B = synth.grid_laplacian_2d(10)
    s = 3.7
    Bs = synth.CSR(B.d, B.row_ptr, B.col, B.val * s)
    r1 = oracle_lib.logdet(B, 0.2, 8.2, 25, 4, seed=9, shift=0.2)
    r2 = oracle_lib.logdet(Bs, 0.2 * s, 8.2 * s, 25, 4, seed=9, shift=0.2 * s)
    assert abs(r2["gamma"] - (r1["gamma"] + B.d * math.log(s))) <= 1e-13 * abs(r2["gamma"])


def test_permutation_invariance(oracle_lib):
    """Gamma(P B P^T) with probes keyed by the original row index equals Gamma(B)."""
    B = synth.random_sparse_spd(50, k_off=3, mseed=3, storage="f64")
    a, b = oracle_lib.gershgorin(B)
    perm = np.random.default_rng(1).permutation(B.d)
    Bp = synth.permute(B, perm)
    m = 5
    V = np.stack([oracle_lib.probe(4, j, B.d) for j in range(m)])
    r1 = oracle_lib.logdet(B, a, b, 20, m, V=V)
    r2 = oracle_lib.logdet(Bp, a, b, 20, m, V=V[:, perm])
    np.testing.assert_allclose(r2["s"], r1["s"], rtol=1e-13)


def test_moment_invariants(oracle_lib):
    """v^T v = d; |v^T T_k(X) v| <= d when spec(X) is in [-1, 1] (|T_k| <= 1 there)."""
    B = synth.grid_laplacian_2d(16)
    r = oracle_lib.logdet(B, 0.1, 8.1, 40, 3, seed=2, shift=0.1, want_moments=True)
    mom = r["moments"]
    assert np.all(mom[:, 0] == B.d)
    assert np.abs(mom).max() <= B.d * (1 + 1e-12)
    # bounds that are too tight (b below lambda_max = 8.1 - eps) push |mu_k| past d
    r = oracle_lib.logdet(B, 0.1, 7.0, 40, 3, seed=2, shift=0.1, want_moments=True)
    assert np.abs(r["moments"]).max() > B.d


def test_negativity_lemma(oracle_lib):
    """Lemma 9: when its condition holds, p_n < 0 on [delta, 1 - delta], so every probe of the
    normalised problem gives a negative v^T p_n(A) v (the lift d log(a+b) removed)."""
    B = synth.random_sparse_spd(80, k_off=2, mseed=8, storage="f64")
    a, b = oracle_lib.gershgorin(B)
    delta = a / (a + b)
    n = next(n for n in range(1, 400)
             if oracle_lib.lemma_bound(delta, n, 1) <= math.log(1.0 / (1.0 - delta)))
    r = oracle_lib.logdet(B, a, b, n, 16, seed=1)
    assert np.all(r["s"] - B.d * math.log(a + b) < 0)


# --------------------------------------------------------------------------------------
# Algorithm 1: statistical pins against closed forms
# --------------------------------------------------------------------------------------

def test_grid32_closed_form_and_cholesky(oracle_lib):
    """the 32x32 grid + 0.1 I (d = 1024): Cholesky log det = closed-form eigen-sum =
    1259.922427278947; E[Gamma] = sum p_30(lambda); over 40 seeds x 50 probes the mean lies
    within 4 sigma of the exact single-probe variance."""
    N, a, b, n, m = 32, 0.1, 8.1, 30, 50
    B = synth.grid_laplacian_2d(N)
    lam = _ref.grid2d_eigs(N) + 0.1
    exact = float(np.log(lam).sum())
    Ld = np.linalg.cholesky(synth.dense(B) + 0.1 * np.eye(B.d))
    assert abs(2 * np.log(np.diag(Ld)).sum() - exact) < 1e-9
    assert abs(exact - 1259.922427278947) < 1e-9
    mean, var = _ref.single_probe_variance_grid2d(N, a, b, n, 0.1)
    assert abs(mean - 1259.922333922736) < 1e-8
    S = 40
    gs = [oracle_lib.logdet(B, a, b, n, m, seed=1000 + s, shift=0.1)["gamma"] for s in range(S)]
    sig = math.sqrt(var / (S * m))
    assert abs(np.mean(gs) - mean) < 4 * sig
    # sample variance of single probes agrees with the exact variance (chi-square, loose)
    r = oracle_lib.logdet(B, a, b, n, 2000, seed=77, shift=0.1)
    assert 0.8 < np.var(r["s"], ddof=1) / var < 1.2


def test_grid3d_gradient_and_value_statistics(oracle_lib):
    """On a small 3-D GMRF Q = tau (kappa^2 I + L): mean of Gamma near sum p_n(lambda);
    mean gradient near the closed-form d/dkappa sum p_n(lambda) = sum p_n'(lambda) 2 tau kappa."""
    N, tau, kappa, n, m = 6, 1.3, 0.4, 40, 64
    L = synth.grid_laplacian_3d(N)
    Q = synth.CSR(L.d, L.row_ptr, L.col, tau * L.val)
    shift = tau * kappa ** 2
    a, b = tau * kappa ** 2, tau * (kappa ** 2 + 12.0)
    lam = tau * (_ref.grid3d_eigs(N) + kappa ** 2)
    e_val = _ref.p_n_on_interval(a, b, n, lam).sum()
    e_dk = (_ref.dp_n_on_interval(a, b, n, lam) * 2 * tau * kappa).sum()
    gs, dks = [], []
    for s in range(12):
        r = oracle_lib.logdet_grad(Q, a, b, n, m, seed=500 + s, shift=shift)
        gs.append(r["gamma"])
        dks.append(r["grad_shift"] * 2 * tau * kappa)
    assert abs(np.mean(gs) - e_val) < 4 * np.std(gs, ddof=1) / math.sqrt(len(gs)) + 1e-9
    assert abs(np.mean(dks) - e_dk) < 4 * np.std(dks, ddof=1) / math.sqrt(len(dks)) + 1e-9
    # closed form derivative of the exact log det, for reference: sum 2 tau kappa / lambda
    assert abs(e_dk - (2 * tau * kappa / lam).sum()) < 1e-3 * abs(e_dk)


def test_theorem1_guarantee(oracle_lib):
    """Theorem 1 as an inequality: with m, n at the theorem's requirement the multiplicative
    error bound holds (probability >= 1 - zeta; here every one of 3 runs)."""
    rng = np.random.default_rng(3)
    d = 40
    Qm, _ = np.linalg.qr(rng.standard_normal((d, d)))
    delta = 0.3
    lam = rng.uniform(delta, 1 - delta, size=d)
    Bd = (Qm * lam) @ Qm.T
    Bd = 0.5 * (Bd + Bd.T)
    rows, cols = np.nonzero(np.ones((d, d)))
    B = synth.CSR(d, np.arange(0, d * d + 1, d, dtype=np.int64), cols.astype(np.int32), Bd[rows, cols])
    eps, zeta = 0.1, 0.2
    m_req, n_req = oracle_lib.thm1_params(eps, zeta, delta)
    m, n = int(math.ceil(m_req)), int(math.ceil(n_req))
    exact = float(np.log(np.linalg.eigvalsh(Bd)).sum())
    # Algorithm 1 input: spectrum in [delta, 1 - delta] means a + b = 1
    for seed in range(3):
        g = oracle_lib.logdet(B, delta, 1 - delta, n, m, seed=seed)["gamma"]
        assert abs(exact - g) <= eps * abs(exact)


def test_theorem2_guarantee(oracle_lib):
    """Theorem 2 as an inequality: C with singular values in [1, sqrt 2] (kappa = sqrt 2), m and n at
    the theorem's requirement for eps = 0.2, zeta = 0.2; |log|det C| - Gamma| <= eps d in every one of
    3 runs (probability >= 1 - zeta each)."""
    rng = np.random.default_rng(8)
    d = 20
    U, _ = np.linalg.qr(rng.standard_normal((d, d)))
    V, _ = np.linalg.qr(rng.standard_normal((d, d)))
    sv = rng.uniform(1.0, math.sqrt(2.0), size=d)
    Cd = (U * sv) @ V.T
    rows, cols = np.nonzero(np.ones((d, d)))
    C = synth.CSR(d, np.arange(0, d * d + 1, d, dtype=np.int64), cols.astype(np.int32), Cd[rows, cols])
    eps, zeta = 0.2, 0.2
    m_req, n_req = oracle_lib.thm2_params(eps, math.sqrt(2.0), zeta)
    m, n = int(math.ceil(m_req)), int(math.ceil(n_req))
    exact = float(np.log(sv).sum())
    assert abs(exact - np.linalg.slogdet(Cd)[1]) < 1e-12
    for seed in range(3):
        g = oracle_lib.logabsdet(C, 1.0, math.sqrt(2.0), n, m, seed=seed)["gamma"]
        assert abs(exact - g) <= eps * d


def test_lemma7_value_on_the_32_grid(oracle_lib):
    """Lemma 7 on the 32x32 grid + 0.1 I with [a, b] = [0.1, 8.1] (delta = a/(a+b)), n = 30, d = 1024:
    the bound evaluates to 5,525 to four figures (an evaluation of the lemma's formula made apart from
    the oracle's code)."""
    assert abs(oracle_lib.lemma_bound(0.1 / 8.2, 30, 1024) - 5525.0) < 0.5


@pytest.mark.parametrize("delta", [0.012195121951219514, 0.05, 0.1, 0.3, 0.45])
def test_lemma7_rate_is_the_ellipse_parameter(oracle_lib, delta):
    """Lemma 7's bound decays by 1/K per degree and grows linearly in d, where K is the sum of
    the semi-axes of the ellipse with foci +-1 and semi-major axis 1/(1 - delta) (Section 4.1,
    Theorem 6): K = 1/(1-delta) + sqrt(1/(1-delta)^2 - 1), the form before the paper simplifies it."""
    ax = 1.0 / (1.0 - delta)
    K = ax + math.sqrt(ax * ax - 1.0)
    for n in (0, 1, 7, 40):
        r = oracle_lib.lemma_bound(delta, n + 1, 5) / oracle_lib.lemma_bound(delta, n, 5)
        assert abs(r - 1.0 / K) < 1e-13
        assert abs(oracle_lib.lemma_bound(delta, n, 14) - 2.0 * oracle_lib.lemma_bound(delta, n, 7)) <= \
            1e-14 * oracle_lib.lemma_bound(delta, n, 14)
    # n = 0: Theorem 6's constant 4M/(K - 1) with M = 5 log(2(1/delta - 1)), per unit of d
    M = 5.0 * math.log(2.0 * (1.0 / delta - 1.0))
    assert abs(oracle_lib.lemma_bound(delta, 0, 1) - 4.0 * M / (K - 1.0)) < 1e-12 * abs(4.0 * M / (K - 1.0))


@pytest.mark.parametrize("eps,zeta,delta", [(0.01, 0.5, 0.1), (0.1, 0.2, 0.3), (0.05, 0.01, 0.02)])
def test_theorem1_requirements_from_the_proof(oracle_lib, eps, zeta, delta):
    """Theorem 1's two requirements, tied to the steps of its proof (Section 4.3):
    the degree is where Lemma 7's bound per unit of d reaches (eps/2) log(1/(1 - delta)) (eq. (3));
    the sample count is Theorem 8's requirement 6 eps0^-2 log(2/zeta0) at eps0 = eps/3 (eq. (4))."""
    m_req, n_req = oracle_lib.thm1_params(eps, zeta, delta)
    assert abs(oracle_lib.lemma_bound(delta, 0, 1) / ((1.0 / ((1.0 / (1.0 - delta)) + math.sqrt(
        (1.0 / (1.0 - delta)) ** 2 - 1.0))) ** -n_req) - eps / 2.0 * math.log(1.0 / (1.0 - delta))) < \
        1e-12 * eps * math.log(1.0 / (1.0 - delta))
    assert abs(m_req - 6.0 / (eps / 3.0) ** 2 * math.log(2.0 / zeta)) < 1e-12 * m_req


@pytest.mark.parametrize("eps,kappa,zeta", [(0.2, math.sqrt(2.0), 0.2), (0.05, 10.0, 0.05), (0.3, 3.0, 0.1)])
def test_theorem2_requirements_from_theorem1(oracle_lib, eps, kappa, zeta):
    """Theorem 2's M and N follow from Theorem 1 applied to B = C^T C/(smin^2 + smax^2), whose
    delta is 1/(1 + kappa^2) and whose |log det B| is at most d log(1 + kappa^2) (its proof):
    N(eps, kappa) is Theorem 1's degree at eps/log(1 + kappa^2), and M(eps, kappa, zeta) is Theorem 1's
    sample count at 2 eps/log(1 + kappa^2), 13.5 log(1 + kappa^2)^2 eps^-2 log(2/zeta), rounded up to 14."""
    Mv, Nv = oracle_lib.thm2_params(eps, kappa, zeta)
    L = math.log(1.0 + kappa ** 2)
    delta = 1.0 / (1.0 + kappa ** 2)
    _, n1 = oracle_lib.thm1_params(eps / L, zeta, delta)
    m1, _ = oracle_lib.thm1_params(2.0 * eps / L, zeta, delta)
    assert abs(Nv - n1) < 1e-12 * abs(n1)
    assert abs(Mv - m1 * 14.0 / 13.5) < 1e-12 * Mv


def test_theorem1_degree_example():
    """Section 3.1 quotes n = 14 for delta = 0.1, eps = 0.01; the printed formula gives 25.95,
    i.e. n = 26 (a discrepancy in the paper, recorded rather than enforced)."""
    import oracle

    _, n_req = oracle.thm1_params(0.01, 0.5, 0.1)
    assert 25.9 < n_req < 26.0


# --------------------------------------------------------------------------------------
# Algorithm 2
# --------------------------------------------------------------------------------------

def test_alg2_per_probe_brute_force(oracle_lib):
    """Algorithm 2 per probe equals (v^T p_n(C^T C / s) v + d log s)/2 with s = smin^2 + smax^2,
    from a dense eigendecomposition of C^T C (not C C^T: a transposed operand fails this)."""
    C = synth.random_nonsingular(30, per_row=4, mseed=2, diag_add=3.0, storage="f64")
    Cd = synth.dense(C)
    sv = np.linalg.svd(Cd, compute_uv=False)
    smin, smax = 0.9 * sv.min(), 1.1 * sv.max()
    n, m = 25, 5
    V = np.stack([np.where(np.arange(C.d) % (j + 2) == 0, -1.0, 1.0) for j in range(m)])
    r = oracle_lib.logabsdet(C, smin, smax, n, m, V=V)
    s = smin ** 2 + smax ** 2
    vals = _ref.brute_probe_values(Cd.T @ Cd, smin ** 2, smax ** 2, n, V)
    # p_n of log on [smin^2, smax^2] already includes log s: Algorithm 2's shift makes it whole
    np.testing.assert_allclose(r["s"], vals / 2.0, rtol=1e-12)
    assert np.isfinite(s)


def test_alg2_statistical_vs_lu(oracle_lib):
    """Algorithm 2 vs dense LU: log|det C| = sum log|U_ii| within the probe standard error."""
    import scipy.linalg

    C = synth.random_nonsingular(200, per_row=3, mseed=9, diag_add=4.0, storage="f64")
    Cd = synth.dense(C)
    lu, piv = scipy.linalg.lu_factor(Cd)
    exact = float(np.log(np.abs(np.diag(lu))).sum())
    sv = np.linalg.svd(Cd, compute_uv=False)
    r = oracle_lib.logabsdet(C, 0.95 * sv.min(), 1.05 * sv.max(), 60, 400, seed=1)
    assert abs(r["gamma"] - exact) < 4 * r["std_err"] + 1e-6 * abs(exact)


def test_alg2_on_spd_matches_alg1_in_expectation(oracle_lib):
    """for SPD C, log|det C| = log det C; Algorithm 2 and Algorithm 1 agree statistically."""
    B = synth.random_sparse_spd(300, k_off=2, mseed=4, storage="f64")
    lam = np.linalg.eigvalsh(synth.dense(B))
    a1, b1 = 0.98 * lam.min(), 1.02 * lam.max()
    r1 = oracle_lib.logdet(B, a1, b1, 40, 400, seed=2)
    r2 = oracle_lib.logabsdet(B, a1, b1, 80, 400, seed=3)
    exact = float(np.log(lam).sum())
    assert abs(r1["gamma"] - exact) < 4 * r1["std_err"]
    assert abs(r2["gamma"] - exact) < 4 * r2["std_err"] + 1e-6 * abs(exact)


# --------------------------------------------------------------------------------------
# Gradient (reverse mode of Algorithm 1)
# --------------------------------------------------------------------------------------

def _transpose_index(B):
    pos = {(int(r), int(c)): t for t, (r, c) in enumerate(zip(B.row_of_entry(), B.col))}
    return np.array([pos[(int(c), int(r))] for r, c in zip(B.row_of_entry(), B.col)])


def test_gradient_vs_central_differences(oracle_lib):
    """central differences of the oracle's own estimate (same probes, a, b fixed).  Moving a
    single stored entry by h changes Gamma by g_t h; moving B_ij and B_ji together changes it by
    (g_ij + g_ji) h = 2 g_ij h, since the gradient of v^T p(B) v is symmetric at symmetric B.  The
    estimate is a polynomial in the entries, so the O(h^2) error is tiny."""
    B = synth.random_sparse_spd(24, k_off=3, mseed=21, storage="f64")
    a, b = oracle_lib.gershgorin(B)
    a, b = 0.9 * a, 1.1 * b
    n, m, seed, shift = 9, 3, 17, 0.05
    g = oracle_lib.logdet_grad(B, a, b, n, m, seed=seed, shift=shift)
    base = oracle_lib.logdet(B, a, b, n, m, seed=seed, shift=shift)["gamma"]
    assert abs(g["gamma"] - base) < 1e-12 * abs(base)
    tr = _transpose_index(B)
    h = 1e-5
    for t in range(0, B.nnz, 7):
        for mirrored in (False, True):
            vp = B.val.copy(); vp[t] += h
            vm = B.val.copy(); vm[t] -= h
            if mirrored and tr[t] != t:
                vp[tr[t]] += h
                vm[tr[t]] -= h
            fp = oracle_lib.logdet(synth.CSR(B.d, B.row_ptr, B.col, vp), a, b, n, m, seed=seed, shift=shift)["gamma"]
            fm = oracle_lib.logdet(synth.CSR(B.d, B.row_ptr, B.col, vm), a, b, n, m, seed=seed, shift=shift)["gamma"]
            fd = (fp - fm) / (2 * h)
            expect = g["grad"][t] * (2.0 if (mirrored and tr[t] != t) else 1.0)
            assert abs(fd - expect) <= 1e-7 * max(1.0, abs(fd)), (t, mirrored)
    # the gradient is symmetric: mirrored entries carry the same value
    np.testing.assert_allclose(g["grad"], g["grad"][tr], rtol=1e-13, atol=0)
    fp = oracle_lib.logdet(B, a, b, n, m, seed=seed, shift=shift + h)["gamma"]
    fm = oracle_lib.logdet(B, a, b, n, m, seed=seed, shift=shift - h)["gamma"]
    assert abs((fp - fm) / (2 * h) - g["grad_shift"]) <= 1e-7 * max(1.0, abs(g["grad_shift"]))


def test_gradient_vs_central_differences_nonsymmetric(oracle_lib):
    """Off the symmetric premise: for a non-symmetric B the recurrence still evaluates
    v^T p(X) v, and its derivative with respect to each stored entry on its own is what central
    differences of the estimate give.  The adjoint recurrence must apply X^T: with X in its
    place the entries of this matrix are off by up to about 200 %."""
    C = synth.random_nonsingular(24, per_row=3, mseed=21, diag_add=3.0, storage="f64")
    a, b, n, m, seed, shift = 0.5, 6.0, 9, 3, 17, 0.05
    g = oracle_lib.logdet_grad(C, a, b, n, m, seed=seed, shift=shift)
    base = oracle_lib.logdet(C, a, b, n, m, seed=seed, shift=shift)["gamma"]
    assert abs(g["gamma"] - base) < 1e-12 * abs(base)
    h = 1e-5
    fds = np.empty(C.nnz)
    for t in range(C.nnz):
        vp = C.val.copy(); vp[t] += h
        vm = C.val.copy(); vm[t] -= h
        fp = oracle_lib.logdet(synth.CSR(C.d, C.row_ptr, C.col, vp), a, b, n, m, seed=seed, shift=shift)["gamma"]
        fm = oracle_lib.logdet(synth.CSR(C.d, C.row_ptr, C.col, vm), a, b, n, m, seed=seed, shift=shift)["gamma"]
        fds[t] = (fp - fm) / (2 * h)
    scale = np.abs(fds).max()
    np.testing.assert_allclose(g["grad"], fds, rtol=1e-6, atol=1e-8 * scale)
    # the matrix really is off the symmetric set
    Cd = synth.dense(C)
    assert np.abs(Cd - Cd.T).max() > 0.5
    fp = oracle_lib.logdet(C, a, b, n, m, seed=seed, shift=shift + h)["gamma"]
    fm = oracle_lib.logdet(C, a, b, n, m, seed=seed, shift=shift - h)["gamma"]
    assert abs((fp - fm) / (2 * h) - g["grad_shift"]) <= 1e-7 * max(1.0, abs(g["grad_shift"]))


def test_gradient_enumeration_nonsymmetric_trace_derivative(oracle_lib):
    """Averaged over all 2^d sign patterns the estimate is tr p_n(B) for any square B, and
    d tr p_n(B)/dB_ij = [p_n'(B)]_ji; for a non-symmetric B that is the transpose of p_n'(B), which
    a dense eigendecomposition (complex eigenvalues, numpy) gives independently."""
    C = synth.random_nonsingular(9, per_row=2, mseed=13, diag_add=3.0, storage="f64")
    Cd = synth.dense(C)
    assert np.abs(Cd - Cd.T).max() > 0.1
    a, b, n = 0.5, 6.0, 7
    V = _ref.all_sign_vectors(C.d)
    g = oracle_lib.logdet_grad(C, a, b, n, V.shape[0], V=V)
    lam, Q = np.linalg.eig(Cd)
    D = ((Q * _ref.dp_n_on_interval(a, b, n, lam)) @ np.linalg.inv(Q)).real
    rows = C.row_of_entry()
    np.testing.assert_allclose(g["grad"], D[C.col, rows], rtol=1e-9, atol=1e-10 * np.abs(D).max())
    assert abs(g["grad_shift"] - np.trace(D)) < 1e-10 * abs(np.trace(D))
    # the transposed reading differs here, so the pin tells the two apart
    assert np.abs(D[C.col, rows] - D[rows, C.col]).max() > 1e-2 * np.abs(D).max()


def test_gradient_enumeration_equals_exact_trace_derivative(oracle_lib):
    """Averaged over all 2^d sign patterns, dGamma/dB_ij = d/dB_ij tr p_n(B) = [p_n'(B)]_ji."""
    B = synth.random_sparse_spd(9, k_off=2, mseed=13, storage="f64")
    Bd = synth.dense(B)
    a, b = oracle_lib.gershgorin(B)
    n = 7
    V = _ref.all_sign_vectors(B.d)
    g = oracle_lib.logdet_grad(B, a, b, n, V.shape[0], V=V)
    D = _ref.pn_matrix(Bd, a, b, n, deriv=True)
    rows = B.row_of_entry()
    np.testing.assert_allclose(g["grad"], D[B.col, rows], rtol=1e-11, atol=1e-12)
    assert abs(g["grad_shift"] - np.trace(D)) < 1e-11 * abs(np.trace(D))


def test_gradient_diagonal_closed_form(oracle_lib):
    """for diagonal B, dGamma/db_ii = p_n'(b_ii) for any probes (numpy chebder)."""
    rng = np.random.default_rng(4)
    a, b, n = 0.3, 6.0, 19
    diag = rng.uniform(a, b, size=33)
    B = synth.diagonal_matrix(diag)
    g = oracle_lib.logdet_grad(B, a, b, n, 2, seed=8)
    np.testing.assert_allclose(g["grad"], _ref.dp_n_on_interval(a, b, n, diag), rtol=1e-12)


def test_gershgorin_interval(oracle_lib):
    """Gershgorin discs (used for the bounds of the random workloads) contain the spectrum."""
    B = synth.random_sparse_spd(200, k_off=4, mseed=1, storage="f32")
    a, b = oracle_lib.gershgorin(B, shift=0.25)
    lam = np.linalg.eigvalsh(synth.dense(B)) + 0.25
    assert a <= lam.min() and lam.max() <= b
    Bd = synth.dense(B)
    off = np.abs(Bd).sum(1) - np.abs(np.diag(Bd))
    assert abs(a - (np.diag(Bd) + 0.25 - off).min()) < 1e-12
    assert abs(b - (np.diag(Bd) + 0.25 + off).max()) < 1e-12

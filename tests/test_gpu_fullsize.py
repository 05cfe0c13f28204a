"""Parity at the full benchmark sizes, in the launch configuration the benchmark uses.

The oracle cannot redo a whole full-size run in test time, so these tests compare outputs it
can compute one at a time: per-probe estimates s_j for sampled probes (each probe is an
independent pass of Algorithm 1), a directional derivative of the gradient (by central
differences of the oracle's estimate along the diagonal shift), and per-matrix estimates
of sampled members of the batch.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests._gpu import U32, dev, entrywise, floor_for, rel, say

pytestmark = pytest.mark.gpu

TOL32 = 1e-4


@pytest.fixture(scope="module")
def ld():
    import torch

    assert torch.cuda.is_available()
    import paper_1503_06394_amd as pkg

    pkg.lib()
    return pkg


def _probe_parity(ld, oracle_lib, B, shift, a, b, n, M, seed, probes, label):
    D = dev(B, shift=shift)
    say(f"full size {label}: GPU forward d={B.d} nnz={B.nnz} M={M} n={n}")
    r = ld.ld_logdet_cheb(D, a, b, n, M, seed, want_probes=True)
    for j in probes:
        say(f"full size {label}: oracle probe {j}")
        o = oracle_lib.logdet(B, a, b, n, 1, seed=seed, ids=np.array([j]), shift=shift)
        assert rel(r["s"][j], o["s"][0], floor_for(a, b, n, B.d, TOL32, U32)) <= TOL32, (label, j, r["s"][j], o["s"][0])
    return r


def test_random_1m_fp32_probes(ld, oracle_lib):
    """d = 1e6 random sparse SPD (Gershgorin bounds), FP32, M = 64 in one block, n = 50."""
    B = synth.random_sparse_spd(1_000_000, 5, 2, 1.0, "f32")
    a, b = oracle_lib.gershgorin(B)
    r = _probe_parity(ld, oracle_lib, B, 0.0, a, b, 50, 64, 2, [0, 37, 63], "random1m")
    assert r["status"] == 0


@pytest.mark.timeout(600)
def test_grid_4096_bf16_probe(ld, oracle_lib):
    """4096 x 4096 Dirichlet grid (d = 16.8M), BF16 values with the 0.01 shift in FP64, FP32
    recurrence, M = 32, n = 100."""
    B = synth.grid_laplacian_2d(4096, "bf16")
    r = _probe_parity(ld, oracle_lib, B, 0.01, 0.01, 8.01, 100, 32, 5, [0], "grid4096")
    assert r["status"] == 0


@pytest.mark.timeout(900)
def test_gmrf_128_fwd_grad(ld, oracle_lib):
    """3-D GMRF 128^3 (d = 2.1M), tau = 1, kappa = 0.3, FP32, M = 32, n = 60: sampled probes of the
    forward, and d Gamma / d shift of the gradient call against central differences of the
    oracle's estimate with the same 32 probes."""
    B = synth.grid_laplacian_3d(128, "f32")
    shift, a, b, n, M, seed = 0.09, 0.09, 12.09, 60, 32, 3
    _probe_parity(ld, oracle_lib, B, shift, a, b, n, M, seed, [0, 31], "gmrf128")
    say("full size gmrf128: GPU gradient")
    r, g = ld.ld_logdet_cheb_grad(dev(B, shift=shift), a, b, n, M, seed)
    # every row stores its diagonal: the diagonal entries of the gradient sum to d/dshift
    rows = B.row_of_entry()
    diag = g.double().cpu().numpy()[B.col == rows].sum()
    assert rel(diag, r["grad_shift"]) <= TOL32
    h = 1e-3
    say("full size gmrf128: oracle central differences along the shift")
    fp = oracle_lib.logdet(B, a, b, n, M, seed=seed, shift=shift + h)["gamma"]
    fm = oracle_lib.logdet(B, a, b, n, M, seed=seed, shift=shift - h)["gamma"]
    fd = (fp - fm) / (2 * h)
    assert rel(r["grad_shift"], fd) <= TOL32, (r["grad_shift"], fd)
    # closed forms of Q = tau (kappa^2 I + L) at tau = 1, kappa = 0.3 from the grid's eigenvalues:
    # d log det Q / d tau = d / tau exactly, and d/d kappa = sum_i 2 kappa / (kappa^2 + lambda_i).
    # The estimator's d/d tau = sum_t g_t L_t + kappa^2 d/d shift has a tiny probe variance (its
    # matrix is p'(Q) Q, close to I); d/d kappa = 2 kappa d/d shift is compared within five times
    # the bound sqrt(2 ||2 kappa p'(Q)||_F^2 / M) on its probe standard error.
    kappa, N = 0.3, 128
    mu = 2.0 - 2.0 * np.cos(np.pi * np.arange(1, N + 1) / (N + 1))
    lam = (mu[:, None, None] + mu[None, :, None] + mu[None, None, :]).ravel()
    dtau = float(g.double().cpu().numpy() @ B.val) + kappa ** 2 * r["grad_shift"]
    assert rel(dtau, float(B.d)) <= 1e-5, dtau
    exact_dk = float((2 * kappa / (kappa ** 2 + lam)).sum())
    se_bound = float(np.sqrt(2 * ((2 * kappa / (kappa ** 2 + lam)) ** 2).sum() / M))
    assert abs(2 * kappa * r["grad_shift"] - exact_dk) <= 5 * se_bound, (2 * kappa * r["grad_shift"], exact_dk)


@pytest.mark.timeout(600)
def test_batch_256_sampled(ld, oracle_lib):
    """256 random SPD matrices, d log-uniform in [1e3, 2e5], 5-20 stored entries per row, own
    Gershgorin bounds and degree n in [20, 80], M = 32, one captured graph; sampled members
    against the oracle."""
    mats = synth.random_batch(256, mseed0=1000)
    ab = [oracle_lib.gershgorin(B) for B in mats]
    ns = [B.meta["n"] for B in mats]
    D = [dev(B) for B in mats]
    say(f"full batch: {len(mats)} matrices, total d={sum(B.d for B in mats)}")
    res = ld.ld_logdet_cheb_batched(D, [x[0] for x in ab], [x[1] for x in ab], ns, 32, 4)
    order = np.argsort([B.d for B in mats])
    for i in [int(order[0]), int(order[1]), int(order[128]), int(order[-1])]:
        say(f"full batch: oracle for member {i} (d={mats[i].d}, n={ns[i]})")
        o = oracle_lib.logdet(mats[i], ab[i][0], ab[i][1], ns[i], 32, seed=4 + i)
        assert rel(res[i]["logdet"], o["gamma"], floor_for(*ab[i], ns[i], mats[i].d, TOL32, U32)) <= TOL32, i


@pytest.mark.timeout(600)
def test_nonsingular_1m_alg2_probe(ld, oracle_lib):
    """Algorithm 2 on the general d = 1e6 matrix (8 N(0,1) entries per row plus 3 I, FP32), M = 32,
    n = 100, bounds from the Lanczos estimate padded as the benchmark pads them; sampled probes."""
    C = synth.random_nonsingular(1_000_000, 8, 6, 3.0, "f32")
    D = dev(C)
    say("full size nonsingular: Lanczos estimate")
    lo, hi = ld.ld_spectral_estimate(D, iters=300, gram=True, seed=6)
    smin, smax = (0.5 * lo) ** 0.5, 1.05 * hi ** 0.5
    say(f"full size nonsingular: GPU Algorithm 2 (smin={smin:.4g}, smax={smax:.4g})")
    r = ld.ld_logabsdet_cheb(D, None, smin, smax, 100, 32, 6, want_probes=True)
    for j in (0, 31):
        say(f"full size nonsingular: oracle probe {j}")
        o = oracle_lib.logabsdet(C, smin, smax, 100, 1, seed=6, ids=np.array([j]))
        assert rel(r["s"][j], o["s"][0], floor_for(smin ** 2, smax ** 2, 100, C.d, TOL32, U32)) <= TOL32, (j, r["s"][j], o["s"][0])


@pytest.mark.timeout(600)
def test_spanning_trees_1m_probe(ld, oracle_lib):
    """Spanning-tree counting on a d = 1e6 hub graph (5 random neighbours drawn per vertex plus the
    hub), Algorithm 2 on L(hub) with sigma in [1, 2 Delta_max - 1], FP32, M = 32, n = 100;
    sampled probes against the oracle's own minor and Algorithm 2."""
    G = synth.hub_graph(1_000_000, 5, 7)
    say("full size spanning trees: GPU minor + Algorithm 2")
    r = ld.ld_log_spanning_trees(dev(G), 0, 100, 32, 8, method=1, want_probes=True)
    for j in (0, 17):
        say(f"full size spanning trees: oracle probe {j}")
        o = oracle_lib.log_spanning_trees(G, 0, 100, 1, seed=8, method=1, ids=np.array([j]))
        assert rel(r["s"][j], o["s"][0], floor_for(1.0, (2.0 * o["delta_max"] - 1.0) ** 2, 100, G.d, TOL32, U32)) <= TOL32, (j, r["s"][j], o["s"][0])


@pytest.mark.timeout(900)
def test_gmrf_5000_likelihood(ld, oracle_lib):
    """The 5000 x 5000 grid GMRF of Section 5.2 (d = 25M): a draw at rho = -0.22, the
    log-likelihood at three values of rho (FP32, M = 16, n = 40, the same probes), maximal at the
    hidden value; probe 0 of the log det at rho = -0.22 against the oracle."""
    import torch

    from paper_1503_06394_amd.gmrf import GMRF

    N = 5000
    say("full size gmrf5000: pattern and sample")
    L = synth.grid_laplacian_2d(N, "f32")
    x = synth.gmrf_sample(N, -0.22, seed=1)
    D = dev(L)
    g = GMRF(D.row_ptr, D.col)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    del D
    say("full size gmrf5000: GPU curve")
    curve = g.sweep([-0.24, -0.22, -0.20], xt, 40, 16, 2)
    assert max(curve, key=lambda r: r["loglik"])["rho"] == -0.22
    J = g.precision(-0.22)
    r = ld.ld_logdet_cheb(J, 0.12, 1.88, 40, 16, 2, want_probes=True)
    del J, g, xt
    say("full size gmrf5000: oracle probe 0")
    Jh = synth.gmrf_grid_precision(N, -0.22, "f32")
    o = oracle_lib.logdet(Jh, 0.12, 1.88, 40, 1, seed=2, ids=np.array([0]))
    assert rel(r["s"][0], o["s"][0], floor_for(0.12, 1.88, 40, Jh.d, TOL32, U32)) <= TOL32


@pytest.mark.timeout(900)
def test_random_1m_gradient_bench_configuration(ld, oracle_lib):
    """The benchmark's fwd+grad call (d = 1e6 random SPD, FP32, M = 64, n = 50, Gershgorin bounds,
    FP32 gradient) against the oracle's gradient averaged over the same 64 probes, computed in CPU
    worker processes: 20000 sampled entries (entry by entry, 1e-4) and d Gamma / d shift (1e-4)."""
    import os

    import torch

    from tests._oracle_pool import mean_gradient

    spec = ("random_sparse_spd", 1_000_000, 5, 2, 1.0, "f32")
    B = synth.random_sparse_spd(*spec[1:])
    D = dev(B)
    a, b = ld.ld_gershgorin(D)
    say("full size random1m gradient: GPU")
    r, g = ld.ld_logdet_cheb_grad(D, a, b, 50, 64, 2, 1.0, grad_dtype=torch.float32)
    idx = np.sort(np.random.default_rng(9).choice(B.nnz, 20_000, replace=False))
    gg = g.double().cpu().numpy()[idx]
    workers = max(1, min(16, (os.cpu_count() or 1)))
    say(f"full size random1m gradient: oracle, 64 probes over {workers} worker processes")
    og, ogs = mean_gradient(spec, a, b, 50, 64, 2, idx, workers)
    assert entrywise(gg, og) <= TOL32
    assert rel(r["grad_shift"], ogs) <= TOL32


@pytest.mark.timeout(900)
def test_gmrf_128_gradient_bench_configuration(ld, oracle_lib):
    """The benchmark's gmrf128 fwd+grad call (128^3 GMRF, FP32, M = 32, n = 60, shift 0.09) against the
    oracle's gradient averaged over the same 32 probes in CPU worker processes: 20000 sampled
    entries (entry by entry, 1e-4) and d Gamma / d shift (1e-4).  The lattice's planes (16384 rows of
    128-byte vector rows) run the general kernels in plane-major tile order."""
    import os

    import torch

    from tests._oracle_pool import mean_gradient

    spec = ("grid_laplacian_3d", 128, "f32")
    B = synth.grid_laplacian_3d(128, "f32")
    shift, a, b, n, M, seed = 0.09, 0.09, 12.09, 60, 32, 3
    say("full size gmrf128 gradient: GPU")
    r, g = ld.ld_logdet_cheb_grad(dev(B, shift=shift), a, b, n, M, seed, 1.0, grad_dtype=torch.float32)
    assert r["plane_tiles"] == 128, r["plane_tiles"]  # 16384-row planes of 128-row tiles
    idx = np.sort(np.random.default_rng(10).choice(B.nnz, 20_000, replace=False))
    gg = g.double().cpu().numpy()[idx]
    workers = max(1, min(16, (os.cpu_count() or 1)))
    say(f"full size gmrf128 gradient: oracle, {M} probes over {workers} worker processes")
    og, ogs = mean_gradient(spec, a, b, n, M, seed, idx, workers, shift=shift)
    assert entrywise(gg, og) <= TOL32
    assert rel(r["grad_shift"], ogs) <= TOL32


@pytest.mark.timeout(900)
def test_grid_4096_gradient_bench_configuration(ld, oracle_lib):
    """The bench's default fwd+grad call (4096^2 grid + 0.01 I, BF16 values with the shift in FP64,
    M = 32, n = 100, FP32 gradient: the staged stencil kernels) against the oracle along one symmetric
    direction through every stored entry and the shift: sum_t g_t e_t + grad_shift e_shift against the
    oracle's forward-mode derivative of the same 32-probe estimate, computed in CPU worker processes
    (the oracle's reverse mode would store 2n + 3 vectors of d doubles per probe).  Relative 1e-4."""
    import os

    import torch

    from tests._oracle_pool import direction, mean_dir

    spec = ("grid_laplacian_2d", 4096, "bf16")
    B = synth.grid_laplacian_2d(4096, "bf16")
    shift, a, b, n, M, seed, dseed = 0.01, 0.01, 8.01, 100, 32, 5, 17
    say("full size grid4096 gradient: GPU")
    r, g = ld.ld_logdet_cheb_grad(dev(B, shift=shift), a, b, n, M, seed, 1.0, grad_dtype=torch.float32)
    assert r["adjoint_form"] == "shifted_staged", r["adjoint_form"]
    e, es = direction(B, dseed)
    gpu = float(np.dot(g.double().cpu().numpy(), e) + r["grad_shift"] * es)
    del g
    workers = max(1, min(16, (os.cpu_count() or 1)))
    say(f"full size grid4096 gradient: oracle directional derivative, {M} probes over {workers} worker processes")
    ora = mean_dir(spec, a, b, n, M, seed, dseed, workers, shift=shift)
    print(f"[grid4096 grad] gpu {gpu:.9e} oracle {ora:.9e} rel {abs(gpu - ora) / abs(ora):.2e}", flush=True)
    assert rel(gpu, ora) <= TOL32

"""Oracle work spread over CPU worker processes for the full-size gradient parity test.

The estimate and its gradient are means over independent probes, so the oracle's per-probe
gradients can be computed in separate processes and summed.  Workers import only numpy, the
input generator and the oracle (never the GPU library); each builds the matrix from its seed and
returns the requested entries of its probes' summed gradients."""
from __future__ import annotations

import numpy as np

_cache = {}


def _matrix(spec):
    if spec not in _cache:
        import synth

        kind, args = spec[0], spec[1:]
        _cache[spec] = {"random_sparse_spd": synth.random_sparse_spd,
                        "grid_laplacian_2d": synth.grid_laplacian_2d,
                        "grid_laplacian_3d": synth.grid_laplacian_3d}[kind](*args)
    return _cache[spec]


def grad_samples(job):
    """job = (matrix spec, shift, a, b, n, seed, probe ids, entry indices): the sum over the given
    probes of the oracle's single-probe gradients at those entries, and of d Gamma / d shift."""
    import oracle

    spec, shift, a, b, n, seed, probes, idx = job
    B = _matrix(spec)
    acc = np.zeros(len(idx))
    gs = 0.0
    for j in probes:
        r = oracle.logdet_grad(B, a, b, n, 1, seed=seed, ids=np.array([j]), shift=shift)
        acc += r["grad"][idx]
        gs += r["grad_shift"]
    return acc, gs


def mean_gradient(spec, a, b, n, M, seed, idx, workers, shift=0.0):
    """Mean over probes 0..M-1 of the oracle's gradient at entries idx, and of d Gamma / d shift.
    spec = (generator name in synth, its arguments...)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    chunks = [list(range(M))[w::workers] for w in range(workers)]
    jobs = [(spec, shift, a, b, n, seed, c, idx) for c in chunks if c]
    # fresh interpreters (never a fork of a process that may hold GPU state); a worker that dies
    # raises BrokenProcessPool instead of being replaced
    with ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(grad_samples, jobs))
    return sum(p[0] for p in parts) / M, sum(p[1] for p in parts) / M


def direction(B, dseed: int):
    """A symmetric direction through every stored entry: e = (rho_i + rho_j)/2 on off-diagonal entries
    (i, j), -rho_i / 2 on diagonal ones, rho ~ U[0.5, 1.5] per row from ``dseed``, and e_shift = 0.25."""
    rho = np.random.default_rng(dseed).uniform(0.5, 1.5, B.d)
    rows = np.repeat(np.arange(B.d), np.diff(B.row_ptr))
    e = 0.5 * (rho[rows] + rho[B.col])
    diag = rows == B.col
    e[diag] = -0.5 * rho[rows[diag]]
    return e, 0.25


def dir_samples(job):
    """job = (matrix spec, shift, a, b, n, seed, probe ids, direction seed): the sum over the given probes
    of the oracle's directional derivative of the single-probe estimate along ``direction``."""
    import oracle

    spec, shift, a, b, n, seed, probes, dseed = job
    B = _matrix(spec)
    e, es = direction(B, dseed)
    return sum(oracle.logdet_dir(B, a, b, n, 1, e, es, seed=seed, ids=np.array([j]), shift=shift) for j in probes)


def mean_dir(spec, a, b, n, M, seed, dseed, workers, shift=0.0):
    """Mean over probes 0..M-1 of the oracle's directional derivative along direction(B, dseed)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    chunks = [list(range(M))[w::workers] for w in range(workers)]
    jobs = [(spec, shift, a, b, n, seed, c, dseed) for c in chunks if c]
    with ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(dir_samples, jobs))
    return sum(parts) / M

"""Small structured test matrices with the patterns that the staged (stencil) kernels take: grids
and lattices in natural order, bands.  Shared by the GPU forward and gradient tests."""
from __future__ import annotations

import numpy as np

import synth


def _grid2d_rect(n1: int, n2: int, storage: str, drop_diag_every: int = 0):
    """Dirichlet 5-point Laplacian on an n1 x n2 grid (node (i, j) = i n2 + j); optionally every
    drop_diag_every-th row without its stored diagonal (the shift carries it)."""
    d = n1 * n2
    idx = np.arange(d)
    i, j = idx // n2, idx % n2
    rows, cols, vals = [], [], []
    for o, m in ((-n2, i > 0), (-1, j > 0), (0, np.ones(d, bool)), (1, j < n2 - 1), (n2, i < n1 - 1)):
        if o == 0 and drop_diag_every:
            m = idx % drop_diag_every != 0
        rows.append(idx[m]), cols.append(idx[m] + o), vals.append(np.full(int(m.sum()), 4.0 if o == 0 else -1.0))
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    order = np.lexsort((c, r))
    rp = np.zeros(d + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=d), out=rp[1:])
    return synth.CSR(d, rp, c[order].astype(np.int32), synth.round_to(v[order], storage), storage)


def _hex2d(n1: int, n2: int, storage: str):
    """7-point (triangular-lattice) Laplacian on an n1 x n2 grid: neighbours (i, j +- 1), (i +- 1, j)
    and (i - 1, j + 1), (i + 1, j - 1); diagonal 6, -1 per in-grid neighbour."""
    d = n1 * n2
    idx = np.arange(d)
    i, j = idx // n2, idx % n2
    rows, cols, vals = [], [], []
    for di, dj in ((-1, 0), (-1, 1), (0, -1), (0, 0), (0, 1), (1, -1), (1, 0)):
        m = (i + di >= 0) & (i + di < n1) & (j + dj >= 0) & (j + dj < n2)
        rows.append(idx[m]), cols.append(idx[m] + di * n2 + dj)
        vals.append(np.full(int(m.sum()), 6.0 if (di, dj) == (0, 0) else -1.0))
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    order = np.lexsort((c, r))
    rp = np.zeros(d + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=d), out=rp[1:])
    return synth.CSR(d, rp, c[order].astype(np.int32), synth.round_to(v[order], storage), storage)


def _banded(d: int, half: int, storage: str, seed: int):
    """Symmetric band matrix (|i - j| <= half) with random off-diagonals and a dominant diagonal."""
    rng = np.random.default_rng(seed)
    A = np.zeros((d, d))
    for k in range(1, half + 1):
        v = rng.uniform(-1.0, 1.0, d - k)
        A[np.arange(d - k), np.arange(k, d)] = v
        A[np.arange(k, d), np.arange(d - k)] = v
    A[np.arange(d), np.arange(d)] = np.abs(A).sum(axis=1) + 1.0
    r, c = np.nonzero(A)
    rp = np.zeros(d + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=d), out=rp[1:])
    return synth.CSR(d, rp, c.astype(np.int32), synth.round_to(A[r, c], storage), storage)

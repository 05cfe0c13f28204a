"""Seeded synthetic sparse matrices for the log-determinant workloads.

This module only builds inputs: CSR patterns and values with the shapes, sizes and
value distributions of the paper's experiments (random sparse symmetric matrices of
Section 5.1, grid GMRF precision matrices of Section 5.2) and of the benchmark
configurations derived from them.  It holds none of the estimator's arithmetic: no
Chebyshev coefficients, no probes, no recurrence and no spectral bounds.  Both the
GPU library's tests and the CPU oracle consume the same arrays.

Every matrix is returned as a :class:`CSR` whose ``val`` array is float64 holding
values that are exactly representable in the declared storage type (``"f64"``,
``"f32"`` or ``"bf16"``), so that a consumer that stores them in that type and a
consumer that keeps them in float64 see identical numbers.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "CSR",
    "round_to",
    "grid_laplacian_2d",
    "grid_laplacian_3d",
    "random_sparse_spd",
    "random_nonsingular",
    "lower_triangular_nonsymmetric",
    "random_batch",
    "diagonal_matrix",
    "graph_from_edges",
    "wheel_graph",
    "complete_graph",
    "hub_graph",
    "gmrf_grid_precision",
    "gmrf_sample",
    "permute",
    "dense",
]


@dataclasses.dataclass
class CSR:
    """Square sparse matrix in CSR form (row-sorted, column-sorted, no duplicates)."""

    d: int
    row_ptr: np.ndarray  # int64, d+1
    col: np.ndarray  # int32, nnz
    val: np.ndarray  # float64, nnz (exact in ``storage``)
    storage: str = "f64"  # "f64" | "f32" | "bf16"
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def row_of_entry(self) -> np.ndarray:
        """Row index of every stored entry (int64, nnz)."""
        return np.repeat(np.arange(self.d, dtype=np.int64), np.diff(self.row_ptr))


def round_to(x: np.ndarray, storage: str) -> np.ndarray:
    """Round float64 values to ``storage`` precision (round-to-nearest-even) and return float64."""
    x = np.asarray(x, dtype=np.float64)
    if storage == "f64":
        return x.copy()
    f = x.astype(np.float32)
    if storage == "f32":
        return f.astype(np.float64)
    if storage == "bf16":
        bits = f.view(np.uint32).astype(np.uint64)
        lsb = (bits >> np.uint64(16)) & np.uint64(1)
        bits = (bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
        return bits.astype(np.uint32).view(np.float32).astype(np.float64)
    raise ValueError(f"unknown storage {storage!r}")


def _from_slots(d: int, cols: np.ndarray, vals: np.ndarray, valid: np.ndarray) -> tuple:
    """Compress a (d, s) slot table whose valid columns are ascending along each row."""
    counts = valid.sum(axis=1).astype(np.int64)
    row_ptr = np.zeros(d + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[valid].astype(np.int32)
    val = vals[valid].astype(np.float64)
    return row_ptr, col, val


def grid_laplacian_2d(N: int, storage: str = "f64") -> CSR:
    """Dirichlet 5-point Laplacian on an N x N grid (diagonal 4, -1 per in-grid neighbour).

    Node (i, j) has index i*N + j.  Eigenvalues are 4 - 2cos(p*pi/(N+1)) - 2cos(q*pi/(N+1)),
    p, q = 1..N, all inside (0, 8).
    """
    d = N * N
    idx = np.arange(d, dtype=np.int64)
    i, j = idx // N, idx % N
    offs = [(-N, i > 0), (-1, j > 0), (0, np.ones(d, bool)), (1, j < N - 1), (N, i < N - 1)]
    cols = np.stack([idx + o for o, _ in offs], axis=1)
    valid = np.stack([m for _, m in offs], axis=1)
    vals = np.where(cols == idx[:, None], 4.0, -1.0)
    row_ptr, col, val = _from_slots(d, cols, vals, valid)
    return CSR(d, row_ptr, col, round_to(val, storage), storage, {"kind": "grid2d", "N": N})


def grid_laplacian_3d(N: int, storage: str = "f64") -> CSR:
    """Dirichlet 7-point Laplacian on an N x N x N grid (diagonal 6, -1 per in-grid neighbour).

    Node (i, j, k) has index (i*N + j)*N + k.  Eigenvalues are
    6 - 2cos(p*pi/(N+1)) - 2cos(q*pi/(N+1)) - 2cos(r*pi/(N+1)), inside (0, 12).
    """
    d = N * N * N
    idx = np.arange(d, dtype=np.int64)
    i, j, k = idx // (N * N), (idx // N) % N, idx % N
    one = np.ones(d, bool)
    offs = [(-N * N, i > 0), (-N, j > 0), (-1, k > 0), (0, one), (1, k < N - 1), (N, j < N - 1), (N * N, i < N - 1)]
    cols = np.stack([idx + o for o, _ in offs], axis=1)
    valid = np.stack([m for _, m in offs], axis=1)
    vals = np.where(cols == idx[:, None], 6.0, -1.0)
    row_ptr, col, val = _from_slots(d, cols, vals, valid)
    return CSR(d, row_ptr, col, round_to(val, storage), storage, {"kind": "grid3d", "N": N})


def _distinct_offdiag_draws(rng: np.random.Generator, d: int, k: int) -> np.ndarray:
    """(d, k) table of distinct column indices per row, uniform over j != i."""
    if k > d - 1:
        raise ValueError("k must be <= d-1")
    rows = np.arange(d, dtype=np.int64)[:, None]
    cand = rng.integers(0, d - 1, size=(d, k), dtype=np.int64)
    cand = cand + (cand >= rows)  # skip the diagonal
    cand.sort(axis=1)
    while True:
        dup = np.zeros_like(cand, dtype=bool)
        dup[:, 1:] = cand[:, 1:] == cand[:, :-1]
        nd = int(dup.sum())
        if nd == 0:
            return cand
        r = np.nonzero(dup)[0]
        new = rng.integers(0, d - 1, size=nd, dtype=np.int64)
        cand[dup] = new + (new >= r)
        cand.sort(axis=1)


def _coo_to_csr(d: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> tuple:
    """Sum duplicates and return row-major, column-sorted CSR arrays."""
    key = rows.astype(np.int64) * d + cols.astype(np.int64)
    uniq, inv = np.unique(key, return_inverse=True)
    summed = np.bincount(inv, weights=vals, minlength=uniq.shape[0])
    r = uniq // d
    c = uniq % d
    counts = np.bincount(r, minlength=d).astype(np.int64)
    row_ptr = np.zeros(d + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, c.astype(np.int32), summed


def _insert_diagonal(d: int, row_ptr, col, val, diag: np.ndarray) -> tuple:
    """Add ``diag`` onto the diagonal, inserting entries where the pattern has none."""
    rows = np.repeat(np.arange(d, dtype=np.int64), np.diff(row_ptr))
    all_rows = np.concatenate([rows, np.arange(d, dtype=np.int64)])
    all_cols = np.concatenate([col.astype(np.int64), np.arange(d, dtype=np.int64)])
    all_vals = np.concatenate([val, diag])
    return _coo_to_csr(d, all_rows, all_cols, all_vals)


def random_sparse_spd(d: int, k_off: int = 5, mseed: int = 2, diag_add: float = 1.0,
                      storage: str = "f32") -> CSR:
    """Random sparse symmetric diagonally dominant matrix (Section 5.1 recipe).

    Each row draws ``k_off`` distinct off-diagonal columns uniformly over j != i with
    values U[-1, 1]; every entry is mirrored to its transposed position and coinciding
    entries are summed (about 2*k_off+1 stored entries per row).  Off-diagonals are
    rounded to ``storage`` first; the diagonal is then sum_j |B_ij| + ``diag_add``,
    summed in float64 over the rounded values and rounded to ``storage``.
    """
    rng = np.random.Generator(np.random.PCG64(mseed))
    cols = _distinct_offdiag_draws(rng, d, k_off)
    vals = rng.uniform(-1.0, 1.0, size=(d, k_off))
    rows = np.repeat(np.arange(d, dtype=np.int64), k_off)
    cflat = cols.reshape(-1)
    vflat = vals.reshape(-1)
    row_ptr, col, val = _coo_to_csr(d, np.concatenate([rows, cflat]), np.concatenate([cflat, rows]),
                                    np.concatenate([vflat, vflat]))
    val = round_to(val, storage)
    rows_e = np.repeat(np.arange(d, dtype=np.int64), np.diff(row_ptr))
    absrow = np.bincount(rows_e, weights=np.abs(val), minlength=d)
    diag = round_to(absrow + diag_add, storage)
    row_ptr, col, val = _insert_diagonal(d, row_ptr, col, val, diag)
    return CSR(d, row_ptr, col, val, storage,
               {"kind": "random_spd", "k_off": k_off, "mseed": mseed, "diag_add": diag_add})


def random_nonsingular(d: int, per_row: int = 8, mseed: int = 6, diag_add: float = 3.0,
                       storage: str = "f32") -> CSR:
    """General (non-symmetric) sparse matrix: ``per_row`` uniform columns per row drawn with
    replacement, N(0, 1) values, duplicates summed, then ``diag_add`` added to C_ii
    (inserted where absent); values rounded to ``storage``."""
    rng = np.random.Generator(np.random.PCG64(mseed))
    cols = rng.integers(0, d, size=(d, per_row), dtype=np.int64)
    vals = rng.standard_normal(size=(d, per_row))
    rows = np.repeat(np.arange(d, dtype=np.int64), per_row)
    row_ptr, col, val = _coo_to_csr(d, rows, cols.reshape(-1), vals.reshape(-1))
    row_ptr, col, val = _insert_diagonal(d, row_ptr, col, val, np.full(d, diag_add))
    return CSR(d, row_ptr, col, round_to(val, storage), storage,
               {"kind": "random_nonsingular", "per_row": per_row, "mseed": mseed, "diag_add": diag_add})


def lower_triangular_nonsymmetric(d: int, per_row: int = 3, mseed: int = 5, diag_lo: float = 10.0,
                                  diag_hi: float = 14.0, off_scale: float = 0.3, storage: str = "f64") -> CSR:
    """Non-symmetric sparse matrix with a real spectrum: diagonal U[diag_lo, diag_hi] plus ``per_row``
    strictly lower-triangular entries per row (columns uniform below the row, duplicates summed),
    N(0, off_scale^2) values.  Its eigenvalues are its diagonal entries, and no stored off-diagonal
    entry has its transpose stored, so its pattern is not symmetric."""
    rng = np.random.Generator(np.random.PCG64(mseed))
    rows = np.repeat(np.arange(d, dtype=np.int64), per_row)
    hi = np.maximum(rows, 1)
    cols = (rng.random(size=rows.shape[0]) * hi).astype(np.int64)
    keep = rows > 0  # row 0 has no entry below the diagonal
    vals = off_scale * rng.standard_normal(size=rows.shape[0])
    row_ptr, col, val = _coo_to_csr(d, rows[keep], cols[keep], vals[keep])
    row_ptr, col, val = _insert_diagonal(d, row_ptr, col, val, rng.uniform(diag_lo, diag_hi, size=d))
    return CSR(d, row_ptr, col, round_to(val, storage), storage,
               {"kind": "lower_triangular_nonsymmetric", "per_row": per_row, "mseed": mseed})


def random_batch(count: int = 256, mseed0: int = 1000, d_min: int = 1000, d_max: int = 200_000,
                 r_min: int = 5, r_max: int = 20, n_min: int = 20, n_max: int = 80,
                 storage: str = "f32") -> list:
    """Batch of random diagonally dominant SPD matrices of uneven size.

    Matrix i uses its own seed ``mseed0 + i``: d log-uniform in [d_min, d_max], a target of
    r in U{r_min..r_max} stored entries per row (ceil((r-1)/2) off-diagonal draws per row before
    mirroring) and a polynomial degree n in U{n_min..n_max} recorded in ``meta["n"]``.
    """
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(mseed0 + i))
        d = int(round(math.exp(rng.uniform(math.log(d_min), math.log(d_max)))))
        r = int(rng.integers(r_min, r_max + 1))
        n = int(rng.integers(n_min, n_max + 1))
        k = max(1, math.ceil((r - 1) / 2))
        B = random_sparse_spd(d, k, mseed=mseed0 + i, diag_add=1.0, storage=storage)
        B.meta.update({"n": n, "r": r, "batch_index": i})
        out.append(B)
    return out


def diagonal_matrix(diag: np.ndarray, storage: str = "f64") -> CSR:
    """Diagonal matrix with the given entries."""
    diag = np.asarray(diag, dtype=np.float64)
    d = diag.shape[0]
    return CSR(d, np.arange(d + 1, dtype=np.int64), np.arange(d, dtype=np.int32), round_to(diag, storage),
               storage, {"kind": "diagonal"})


def permute(B: CSR, perm: np.ndarray) -> CSR:
    """Return P B P^T, where new row r is old row perm[r]."""
    perm = np.asarray(perm, dtype=np.int64)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(B.d, dtype=np.int64)
    rows = B.row_of_entry()
    new_rows = inv[rows]
    new_cols = inv[B.col.astype(np.int64)]
    row_ptr, col, val = _coo_to_csr(B.d, new_rows, new_cols, B.val)
    return CSR(B.d, row_ptr, col, val, B.storage, dict(B.meta, permuted=True))


def dense(B: CSR) -> np.ndarray:
    """Dense float64 copy (small matrices only)."""
    A = np.zeros((B.d, B.d))
    A[B.row_of_entry(), B.col.astype(np.int64)] = B.val
    return A


# ----------------------------------------------------------------------------------------
# graphs for spanning-tree counting (adjacency patterns, values 1)


def graph_from_edges(nv: int, u: np.ndarray, v: np.ndarray, kind: str = "graph") -> CSR:
    """Adjacency pattern of the simple undirected graph on ``nv`` vertices with edges (u[e], v[e]):
    both orientations stored, repeated edges merged, self loops dropped, columns sorted, values 1."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    rows = np.concatenate([u[keep], v[keep]])
    cols = np.concatenate([v[keep], u[keep]])
    key = np.unique(rows * nv + cols)
    r, c = key // nv, key % nv
    row_ptr = np.zeros(nv + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=nv), out=row_ptr[1:])
    return CSR(nv, row_ptr, c.astype(np.int32), np.ones(key.shape[0]), "f32", {"kind": kind})


def wheel_graph(k: int) -> CSR:
    """Wheel W_k: hub 0 joined to every vertex of the cycle 1..k (k >= 3)."""
    if k < 3:
        raise ValueError("a wheel needs a cycle of at least 3 vertices")
    ring = np.arange(1, k + 1, dtype=np.int64)
    u = np.concatenate([np.zeros(k, dtype=np.int64), ring])
    v = np.concatenate([ring, np.roll(ring, -1)])
    return graph_from_edges(k + 1, u, v, "wheel")


def complete_graph(nv: int) -> CSR:
    """Complete graph K_nv."""
    iu, ju = np.triu_indices(nv, 1)
    return graph_from_edges(nv, iu, ju, "complete")


def hub_graph(nv: int, k_off: int = 5, mseed: int = 7) -> CSR:
    """Vertex 0 joined to every other vertex, plus ``k_off`` distinct uniform random neighbours
    drawn for each of the vertices 1..nv-1 among the others (edges mirrored and merged), so that
    non-hub degrees are about 2 k_off + 1.  The class of graphs of the spanning-tree section."""
    rng = np.random.default_rng(mseed)
    m = nv - 1
    draws = _distinct_offdiag_draws(rng, m, k_off) + 1  # among vertices 1..nv-1
    u = np.concatenate([np.zeros(m, dtype=np.int64), np.repeat(np.arange(1, nv, dtype=np.int64), k_off)])
    v = np.concatenate([np.arange(1, nv, dtype=np.int64), draws.reshape(-1)])
    return graph_from_edges(nv, u, v, "hub")


# ----------------------------------------------------------------------------------------
# grid GMRF with partial correlation rho (maximum-likelihood experiment of Section 5.2)


def gmrf_grid_precision(N: int, rho: float, storage: str = "f32") -> CSR:
    """Precision matrix J(rho) of the N x N grid GMRF whose nodes have four neighbours with
    partial correlation rho: J_ii = 1 and J_ij = -rho for grid neighbours (Dirichlet boundary, so
    border nodes have fewer neighbours).  Positive definite for |rho| < 1/4."""
    L = grid_laplacian_2d(N, "f64")
    diag = L.col.astype(np.int64) == L.row_of_entry()
    val = np.where(diag, 1.0, -float(rho))
    return CSR(L.d, L.row_ptr, L.col, round_to(val, storage), storage, {"kind": "gmrf_grid", "N": N, "rho": rho})


def gmrf_sample(N: int, rho: float, seed: int = 0, z: np.ndarray | None = None) -> np.ndarray:
    """One exact draw x ~ N(0, J(rho)^{-1}) of the grid GMRF above (float64, length N*N), with
    J(rho) taken in exact arithmetic.  The grid's adjacency matrix is diagonalised by the
    orthonormal type-I discrete sine transform S (S = S^T = S^{-1}, eigenvalues
    2cos(p pi/(N+1)) + 2cos(q pi/(N+1))), so x = S diag(1 - rho lambda_pq)^{-1/2} S z with z
    standard normal (drawn from ``seed`` unless given as an (N*N,) or (N*N, k) array)."""
    from scipy.fft import dstn

    if z is None:
        z = np.random.default_rng(seed).standard_normal(N * N)
    z = np.asarray(z, dtype=np.float64)
    cols = z.reshape(N * N, -1)
    t = np.pi * np.arange(1, N + 1) / (N + 1)
    lam = 2.0 * np.cos(t)[:, None] + 2.0 * np.cos(t)[None, :]
    scale = 1.0 / np.sqrt(1.0 - rho * lam)
    out = np.empty_like(cols)
    for k in range(cols.shape[1]):
        g = dstn(cols[:, k].reshape(N, N), type=1, norm="ortho")
        out[:, k] = dstn(g * scale, type=1, norm="ortho").reshape(-1)
    return out.reshape(z.shape)

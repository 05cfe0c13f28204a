"""Oracle for the stochastic Chebyshev log-determinant estimator (arXiv 1503.06394).

TEST INFRASTRUCTURE ONLY.  A ctypes binding to ``liboracle.so`` (plain single-threaded
FP64 C built from ``ldo.c``) plus a few small numpy helpers.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import this package; the GPU
library never does, and this package never imports the GPU library.

Parity status: every function here is pinned by the CPU test suite (closed forms,
library routines, brute force), except those whose docstring says "parity unpinned".
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LDO_SANITIZE=1 selects the AddressSanitizer/UBSan build (see make_lib.py for the command line).
SANITIZE = os.environ.get("LDO_SANITIZE", "0") == "1"
LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")

_lib = None


class _Csr(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
    ]


class _Probes(ctypes.Structure):
    _fields_ = [("V", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("ids", ctypes.c_void_p)]


def build(verbose: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (plain C99, -O2, no fast-math), or the sanitizer build
    ``liboracle_san.so`` when LDO_SANITIZE=1."""
    from .make_lib import build as _build

    return _build(verbose=verbose, sanitize=SANITIZE)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P, D, I, I64, U64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        L.ldo_cheb_nodes.argtypes = [I, P]
        L.ldo_cheb_coeffs_from_values.argtypes = [I, P, P]
        L.ldo_cheb_coeffs_alg1.argtypes = [D, I, P]
        L.ldo_probe_sign.argtypes = [U64, I64, I64]
        L.ldo_probe.argtypes = [U64, I64, I64, P]
        L.ldo_logdet.argtypes = [P, D, D, D, I, I, P, P, P, P]
        L.ldo_logabsdet.argtypes = [P, D, D, I, I, P, P, P]
        L.ldo_logdet_grad.argtypes = [P, D, D, D, I, I, P, P, P, P]
        L.ldo_logdet_dir.argtypes = [P, D, D, D, I, I, P, P, D, P]
        L.ldo_gershgorin.argtypes = [P, D, P, P]
        L.ldo_logdet_taylor.argtypes = [P, D, D, D, I, I, P, P, P]
        L.ldo_lemma_bound.argtypes = [D, I, I64]
        L.ldo_lemma_bound.restype = D
        for f in ("ldo_cheb_coeffs_alg1", "ldo_probe_sign", "ldo_logdet", "ldo_logabsdet",
                  "ldo_logdet_grad", "ldo_logdet_dir", "ldo_gershgorin", "ldo_logdet_taylor"):
            getattr(L, f).restype = I
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class _Keep:
    """Holds numpy arrays alive while a ctypes struct points at them."""

    def __init__(self, B):
        self.row_ptr = np.ascontiguousarray(B.row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(B.col, dtype=np.int32)
        self.val = np.ascontiguousarray(B.val, dtype=np.float64)
        self.s = _Csr(int(B.d), int(self.col.shape[0]), _ptr(self.row_ptr).value, _ptr(self.col).value,
                      _ptr(self.val).value)


def _probes(seed, V, ids, d, m):
    keep = []
    if V is not None:
        V = np.ascontiguousarray(V, dtype=np.float64)
        if V.shape != (m, d):
            raise ValueError(f"V must have shape (m, d) = {(m, d)}, got {V.shape}")
        keep.append(V)
        return _Probes(_ptr(V).value, 0, None), keep
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        if ids.shape != (m,):
            raise ValueError("ids must have shape (m,)")
        keep.append(ids)
        return _Probes(None, int(seed) & (2**64 - 1), _ptr(ids).value), keep
    return _Probes(None, int(seed) & (2**64 - 1), None), keep


def cheb_nodes(n: int) -> np.ndarray:
    x = np.empty(n + 1)
    lib().ldo_cheb_nodes(n, _ptr(x))
    return x


def cheb_coeffs_from_values(fx) -> np.ndarray:
    fx = np.ascontiguousarray(fx, dtype=np.float64)
    c = np.empty_like(fx)
    lib().ldo_cheb_coeffs_from_values(fx.shape[0] - 1, _ptr(fx), _ptr(c))
    return c


def cheb_coeffs_alg1(delta: float, n: int) -> np.ndarray:
    """Coefficients of log(1 - ((1-2 delta)x + 1)/2) on [-1, 1] (Algorithm 1)."""
    c = np.empty(n + 1)
    if lib().ldo_cheb_coeffs_alg1(float(delta), int(n), _ptr(c)):
        raise ValueError("invalid delta or n")
    return c


def probe_sign(seed: int, j: int, r: int) -> int:
    return int(lib().ldo_probe_sign(int(seed) & (2**64 - 1), int(j), int(r)))


def probe(seed: int, j: int, d: int) -> np.ndarray:
    v = np.empty(d)
    lib().ldo_probe(int(seed) & (2**64 - 1), int(j), int(d), _ptr(v))
    return v


def logdet(B, a: float, b: float, n: int, m: int, seed: int = 0, V=None, ids=None, shift: float = 0.0,
           want_moments: bool = False) -> dict:
    """log det(B + shift I) by Algorithm 1 on (B + shift I)/(a+b) plus d log(a+b).

    Returns dict(gamma, s[m], std_err, moments[m, n+1] (A-form moments v^T T_k(X) v) if asked).
    """
    k = _Keep(B)
    pr, keep = _probes(seed, V, ids, B.d, m)
    g = ctypes.c_double(0.0)
    s = np.empty(m)
    mom = np.empty((m, n + 1)) if want_moments else None
    rc = lib().ldo_logdet(ctypes.byref(k.s), float(shift), float(a), float(b), int(n), int(m), ctypes.byref(pr),
                          ctypes.byref(g), _ptr(s), _ptr(mom) if mom is not None else None)
    if rc:
        raise ValueError(f"ldo_logdet failed ({rc})")
    out = {"gamma": g.value, "s": s, "std_err": float(np.std(s, ddof=1) / math.sqrt(m)) if m > 1 else float("nan")}
    if mom is not None:
        out["moments"] = mom
    return out


def logabsdet(C, smin: float, smax: float, n: int, m: int, seed: int = 0, V=None, ids=None) -> dict:
    """log|det C| by Algorithm 2."""
    k = _Keep(C)
    pr, keep = _probes(seed, V, ids, C.d, m)
    g = ctypes.c_double(0.0)
    s = np.empty(m)
    rc = lib().ldo_logabsdet(ctypes.byref(k.s), float(smin), float(smax), int(n), int(m), ctypes.byref(pr),
                             ctypes.byref(g), _ptr(s))
    if rc:
        raise ValueError(f"ldo_logabsdet failed ({rc})")
    return {"gamma": g.value, "s": s, "std_err": float(np.std(s, ddof=1) / math.sqrt(m)) if m > 1 else float("nan")}


def logdet_taylor(B, a: float, b: float, n: int, m: int, seed: int = 0, V=None, ids=None,
                  shift: float = 0.0) -> dict:
    """Taylor-series comparator of Section 5.1's accuracy comparison: d log(a + b) minus the
    degree-n truncation of sum_k tr(A^k)/k, A = I - (B + shift I)/(a + b), traces by the probes."""
    k = _Keep(B)
    pr, keep = _probes(seed, V, ids, B.d, m)
    g = ctypes.c_double(0.0)
    s = np.empty(m)
    rc = lib().ldo_logdet_taylor(ctypes.byref(k.s), float(shift), float(a), float(b), int(n), int(m),
                                 ctypes.byref(pr), ctypes.byref(g), _ptr(s))
    if rc:
        raise ValueError(f"ldo_logdet_taylor failed ({rc})")
    return {"gamma": g.value, "s": s, "std_err": float(np.std(s, ddof=1) / math.sqrt(m)) if m > 1 else float("nan")}


def logdet_grad(B, a: float, b: float, n: int, m: int, seed: int = 0, V=None, ids=None, shift: float = 0.0) -> dict:
    """Gradient of the ``logdet`` estimate w.r.t. the stored entries of B and the diagonal shift."""
    k = _Keep(B)
    pr, keep = _probes(seed, V, ids, B.d, m)
    grad = np.empty(B.nnz)
    gs = ctypes.c_double(0.0)
    g = ctypes.c_double(0.0)
    rc = lib().ldo_logdet_grad(ctypes.byref(k.s), float(shift), float(a), float(b), int(n), int(m),
                               ctypes.byref(pr), _ptr(grad), ctypes.byref(gs), ctypes.byref(g))
    if rc:
        raise ValueError(f"ldo_logdet_grad failed ({rc})")
    return {"gamma": g.value, "grad": grad, "grad_shift": gs.value}


def logdet_dir(B, a: float, b: float, n: int, m: int, e_val, e_shift: float = 0.0, seed: int = 0, V=None, ids=None,
               shift: float = 0.0) -> float:
    """Directional derivative of the ``logdet`` estimate along B -> B + h E (forward mode): E has the
    values ``e_val`` on B's pattern and ``e_shift`` on the diagonal."""
    k = _Keep(B)
    pr, keep = _probes(seed, V, ids, B.d, m)
    e = np.ascontiguousarray(e_val, dtype=np.float64)
    if e.shape != (B.nnz,):
        raise ValueError("e_val must hold one value per stored entry")
    out = ctypes.c_double(0.0)
    rc = lib().ldo_logdet_dir(ctypes.byref(k.s), float(shift), float(a), float(b), int(n), int(m),
                              ctypes.byref(pr), _ptr(e), float(e_shift), ctypes.byref(out))
    if rc:
        raise ValueError(f"ldo_logdet_dir failed ({rc})")
    return out.value


def gershgorin(B, shift: float = 0.0) -> tuple:
    k = _Keep(B)
    a = ctypes.c_double(0.0)
    b = ctypes.c_double(0.0)
    if lib().ldo_gershgorin(ctypes.byref(k.s), float(shift), ctypes.byref(a), ctypes.byref(b)):
        raise ValueError("ldo_gershgorin failed")
    return a.value, b.value


def lemma_bound(delta: float, n: int, d: int) -> float:
    """Lemma 7 right-hand side."""
    return float(lib().ldo_lemma_bound(float(delta), int(n), int(d)))


def thm1_params(eps: float, zeta: float, delta: float) -> tuple:
    """Sample count and degree required by Theorem 1: (m_min, n_min) as real numbers."""
    m = 54.0 / eps ** 2 * math.log(2.0 / zeta)
    K = (math.sqrt(2 - delta) + math.sqrt(delta)) / (math.sqrt(2 - delta) - math.sqrt(delta))
    num = math.log(20.0 / eps * (math.sqrt(2.0 / delta - 1.0) - 1.0) * math.log(2.0 * (1.0 / delta - 1.0))
                   / math.log(1.0 / (1.0 - delta)))
    return m, num / math.log(K)


def thm2_params(eps: float, kappa: float, zeta: float) -> tuple:
    """(M(eps, kappa, zeta), N(eps, kappa)) of Theorem 2."""
    Mv = 14.0 / eps ** 2 * math.log(1 + kappa ** 2) ** 2 * math.log(2.0 / zeta)
    q = math.sqrt(2 * kappa ** 2 + 1)
    num = math.log(20.0 / eps * (q - 1) * math.log(1 + kappa ** 2) * math.log(2 * kappa ** 2)
                   / math.log(1 + kappa ** -2))
    return Mv, num / math.log((q + 1) / (q - 1))


def logdet_batch(mats, a, b, ns, m: int, seed0: int, shift=None) -> list:
    """Batched form: matrix i uses probe seed seed0 + i, its own [a_i, b_i] and degree n_i."""
    out = []
    for i, B in enumerate(mats):
        out.append(logdet(B, a[i], b[i], ns[i], m, seed=seed0 + i, shift=0.0 if shift is None else shift[i]))
    return out


class SimpleCsr:
    """Plain CSR container (row_ptr int64, col int32, val float64) for matrices the oracle builds."""

    def __init__(self, d, row_ptr, col, val):
        self.d = int(d)
        self.row_ptr = np.asarray(row_ptr, dtype=np.int64)
        self.col = np.asarray(col, dtype=np.int32)
        self.val = np.asarray(val, dtype=np.float64)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def laplacian_minor(adj, hub: int) -> tuple:
    """Kirchhoff's matrix-tree theorem (Section 3.3): the Laplacian L = D - A of the graph with
    adjacency pattern ``adj`` (both orientations of every edge stored), with the row and column
    of vertex ``hub`` deleted.  Returns (minor as SimpleCsr with sorted columns, Delta_max), where
    Delta_max is the largest degree among the vertices other than the hub."""
    d = int(adj.d)
    row_ptr = np.asarray(adj.row_ptr, dtype=np.int64)
    deg = np.diff(row_ptr)
    entries = {}
    for r in range(d):
        if r == hub:
            continue
        rr = r - (1 if r > hub else 0)
        row = {rr: float(deg[r])}
        for t in range(row_ptr[r], row_ptr[r + 1]):
            c = int(adj.col[t])
            if c == hub or c == r:
                continue
            cc = c - (1 if c > hub else 0)
            row[cc] = row.get(cc, 0.0) - 1.0
        entries[rr] = sorted(row.items())
    m = d - 1
    rp = np.zeros(m + 1, dtype=np.int64)
    cols, vals = [], []
    for rr in range(m):
        rp[rr + 1] = rp[rr] + len(entries[rr])
        for c, v in entries[rr]:
            cols.append(c)
            vals.append(v)
    others = np.delete(deg, hub)
    return SimpleCsr(m, rp, cols, vals), int(others.max()) if others.size else 0


def log_spanning_trees(adj, hub: int, n: int, m: int, seed: int = 0, method: int = 1, V=None, ids=None) -> dict:
    """Estimate of log tau(G) for a graph whose vertex ``hub`` is adjacent to every other vertex
    (Section 3.3): the spectrum of L(hub) lies in [1, 2 Delta_max - 1], so method 1 runs
    Algorithm 2 with C = L(hub) and singular values in that interval (the corollary's inputs),
    and method 0 runs Algorithm 1 on L(hub) with that interval.  Delta_max = 1 means L(hub) = I,
    and log tau = 0 exactly."""
    L, dmax = laplacian_minor(adj, hub)
    if dmax <= 1:
        return {"gamma": 0.0, "s": np.zeros(m), "minor": L, "delta_max": dmax}
    hi = 2.0 * dmax - 1.0
    if method == 1:
        r = logabsdet(L, 1.0, hi, n, m, seed=seed, V=V, ids=ids)
    else:
        r = logdet(L, 1.0, hi, n, m, seed=seed, V=V, ids=ids)
    r["minor"] = L
    r["delta_max"] = dmax
    return r


def lanczos_extremes(B, iters: int, seed: int = 0, shift: float = 0.0, gram: bool = False) -> tuple:
    """Estimates of the extreme eigenvalues of B + shift I (gram False, B symmetric) or of C^T C
    (gram True, C = B): the extreme Ritz values after ``iters`` steps of the Lanczos process in FP64
    without reorthogonalisation, started from probe 0 of ``seed`` scaled to unit length.  Section 3.2
    asks for bounds on the extreme eigenvalues (singular values) and points to power-type
    iteration; the Lanczos process is the Krylov method that converges fastest to both ends at once.
    Returns (lo, hi, alphas, betas): the smallest and largest eigenvalue of the tridiagonal matrix
    T with diagonal alphas and off-diagonal betas."""
    d = int(B.d)
    rows = np.repeat(np.arange(d), np.diff(np.asarray(B.row_ptr)))
    col = np.asarray(B.col, dtype=np.int64)
    val = np.asarray(B.val, dtype=np.float64)

    def apply(x):  # B x, or C^T (C x)
        y = np.bincount(rows, weights=val * x[col], minlength=d)
        if gram:
            return np.bincount(col, weights=val * y[rows], minlength=d)
        return y + shift * x

    v = probe(seed, 0, d) / math.sqrt(d)
    v_prev = np.zeros(d)
    beta = 0.0
    alphas, betas = [], []
    for j in range(iters):
        w = apply(v)
        alpha = float(w @ v)
        w = w - alpha * v - beta * v_prev
        alphas.append(alpha)
        bb = float(w @ w)
        if not (bb > 0.0 and math.isfinite(bb)):
            break  # the Krylov space is invariant
        beta = math.sqrt(bb)
        if j + 1 < iters:
            betas.append(beta)
        v_prev, v = v, w / beta
    betas = betas[:len(alphas) - 1]
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1]), np.array(alphas), np.array(betas)

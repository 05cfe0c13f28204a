"""Helpers shared by the GPU parity tests: device upload and comparison with the oracle."""
from __future__ import annotations

import math
import sys

import numpy as np


U64 = 2.0 ** -53  # unit roundoff of FP64
U32 = 2.0 ** -24  # unit roundoff of FP32


def floor_for(a: float, b: float, n: int, d: int, tol: float, u: float = U64) -> float:
    """Floor of the denominator of a relative parity check on a log det estimate: E / tol, with E the
    rounding the two sides may commit in Gamma = sum_k c_k mu_k.  Two sources:
      * a moment |mu_k| <= d comes out of k steps of the recurrence with about (k + 1) u d of
        rounding (u the unit roundoff of the recurrence) and c_k weighs it: 2 u d sum_k (k + 1) |c_k|
        per side;
      * each side computes the c_k itself, in FP64, as a sum of n + 1 terms (2/(n+1)) f(x_j) cos(.)
        with |f| <= F = max(|log a|, |log b|): |dc_k| <= 2 (n + 1) u64 F, which |mu_k| <= d carries
        into Gamma as 2 (n + 1)^2 u64 d F per side.
    E = 2 x (both), with a factor 2 of margin on the first.  The check |x - y| / max(|y|, E / tol) <= tol
    passes when |x - y| <= max(tol |y|, E): relative while |Gamma| is above the rounding scale,
    absolute at that scale below it (at 1e-10 the floor is ~1e-12 d for the configurations' degrees,
    far below their |Gamma| / d >= 1)."""
    from tests import _ref

    c = _ref.cheb_coeffs(a, b, n)
    k = np.arange(n + 1)
    F = max(abs(math.log(a)), abs(math.log(b)))
    rec = 4.0 * u * d * float(np.sum((k + 1) * np.abs(c)))
    coef = 4.0 * (n + 1) ** 2 * U64 * d * F
    return (rec + coef) / tol


def floor_taylor(a: float, b: float, n: int, d: int, tol: float, u: float = U64) -> float:
    """floor_for for the Taylor comparator: its terms v^T A^k v / k have |A| <= q = b/(a + b), so a term
    carries about (k + 1) u d q^k / k of rounding; E = 4 u d sum_{k=1..n} (k + 1) q^k / k."""
    q = b / (a + b)
    k = np.arange(1, n + 1)
    return 4.0 * u * d * float(np.sum((k + 1) * q ** k / k)) / tol


def say(msg: str) -> None:
    """Name the case before any GPU work, so a failing run says what it was doing."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(B, dtype=None, shift=0.0):
    import paper_1503_06394_amd as ld

    return ld.DeviceCSR.from_host(B, dtype=dtype, diag_shift=shift)


def rel(x, y, floor=0.0) -> float:
    return abs(x - y) / max(abs(y), floor)


# Gradients are compared entry by entry: |g_t - o_t| <= tol * max(|o_t|, TAU * max_s |o_s|).  An entry
# far below the largest is held to that absolute level instead of its own relative one, because its
# value is a sum (over probes and degrees) of terms as large as those of the large entries, and its
# rounding error scales with those terms, not with the sum.
TAU = 1e-2


def entrywise(g, ref, tau: float = TAU) -> float:
    """max_t |g_t - ref_t| / max(|ref_t|, tau * max|ref|): the entrywise relative error with a floor."""
    g = np.asarray(g, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    if ref.size == 0:
        return 0.0
    den = np.maximum(np.abs(ref), tau * max(float(np.max(np.abs(ref))), 1e-300))
    err = float(np.max(np.abs(g - ref) / den))
    print(f"[entrywise] {err:.3e} over {ref.size} entries", flush=True)
    return err


def normwise(x, y) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300))


def b_form_moments(oracle_moments: np.ndarray) -> np.ndarray:
    """The oracle's Algorithm 1 runs on X = -At (A = I - B form); its moments v^T T_k(X) v equal
    (-1)^k v^T T_k(At) v, the GPU library's moments."""
    k = np.arange(oracle_moments.shape[1])
    return oracle_moments * ((-1.0) ** k)[None, :]

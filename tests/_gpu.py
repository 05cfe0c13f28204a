"""Helpers shared by the GPU parity tests: device upload and comparison with the oracle."""
from __future__ import annotations

import sys

import numpy as np


# Relative errors of log det estimates use max(|reference|, FLOOR * d) as denominator: a log det
# within 1e-3 d of zero is compared in absolute terms, because the FP64 rounding of the final
# coefficient sum scales with d, not with |log det|.
FLOOR = 1e-3


def say(msg: str) -> None:
    """Name the case before any GPU work, so a failing run says what it was doing."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(B, dtype=None, shift=0.0):
    import paper_1503_06394_amd as ld

    return ld.DeviceCSR.from_host(B, dtype=dtype, diag_shift=shift)


def rel(x, y, floor=0.0) -> float:
    return abs(x - y) / max(abs(y), floor)


def normwise(x, y) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300))


def b_form_moments(oracle_moments: np.ndarray) -> np.ndarray:
    """The oracle's Algorithm 1 runs on X = -At (A = I - B form); its moments v^T T_k(X) v equal
    (-1)^k v^T T_k(At) v, the GPU library's moments."""
    k = np.arange(oracle_moments.shape[1])
    return oracle_moments * ((-1.0) ** k)[None, :]

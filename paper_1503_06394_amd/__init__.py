"""Python binding of liblogdet_cheb, the MI355X stochastic Chebyshev log-determinant library.

Method: Han, Malioutov & Shin, "Large-scale Log-determinant Computation through Stochastic
Chebyshev Expansions" (arXiv 1503.06394), Algorithms 1 and 2.

This module only marshals arguments: it turns torch device tensors into the plain pointers
of the C ABI (include/logdet_cheb.h) and calls the shared library, whose HIP kernels run
every step of the estimator.  PyTorch supplies device memory and the current stream.  There
is no CPU fallback: if the library is not built, every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import torch

__all__ = [
    "LogdetChebError", "DeviceCSR", "lib", "ld_logdet_cheb", "ld_logdet_cheb_noalloc", "ld_logabsdet_cheb", "ld_logdet_cheb_grad",
    "ld_logdet_cheb_batched", "ld_gershgorin", "ld_probes", "ld_transpose", "ld_workspace_bytes", "ld_copy",
    "ld_version", "ld_clear_cache", "ld_spectral_estimate", "ld_laplacian_minor", "ld_log_spanning_trees",
    "ld_logdet_taylor", "ld_quadratic_form", "ld_gershgorin_batched",
    "LogdetCheb", "logdet_cheb", "logdet", "as_device_csr", "LD_F64", "LD_F32", "LD_BF16", "LD_WBOUNDS",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblogdet_cheb.so")

LD_F64, LD_F32, LD_BF16 = 0, 1, 2
LD_WBOUNDS = 1
_DTYPE = {torch.float64: LD_F64, torch.float32: LD_F32, torch.bfloat16: LD_BF16}


_ADJ_FORMS = {0: None, 1: "explicit_single", 2: "explicit_two", 3: "shifted", 4: "plain", 5: "shifted_staged"}


class LogdetChebError(RuntimeError):
    pass


class _CSR(ctypes.Structure):
    _fields_ = [
        ("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("values", ctypes.c_void_p),
        ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32), ("diag_shift", ctypes.c_double),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("logdet", ctypes.c_double), ("std_err", ctypes.c_double), ("poly_bound", ctypes.c_double),
        ("grad_shift", ctypes.c_double), ("kernel_ms", ctypes.c_double), ("adjoint_ms", ctypes.c_double),
        ("kernel_launches", ctypes.c_int32), ("adjoint_launches", ctypes.c_int32),
        ("n", ctypes.c_int32), ("M", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("adjoint_form", ctypes.c_int32), ("plane_tiles", ctypes.c_int32),
        ("staged_steps", ctypes.c_int32),
    ]


class _Opts(ctypes.Structure):
    _fields_ = [
        ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t), ("vec_f64", ctypes.c_int32),
        ("ckpt_stride", ctypes.c_int32), ("tile", ctypes.c_int32), ("probe_tile", ctypes.c_int32),
        ("timing", ctypes.c_int32), ("plain_recurrence", ctypes.c_int32),
        ("moments_out", ctypes.c_void_p), ("probe_out", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """Load liblogdet_cheb.so (built in-tree by __graft_entry__.build()); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LogdetChebError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        P, D, I, I64, U64, SZ = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.c_size_t)
        L.ld_logdet_cheb.argtypes = [P, D, D, I, I, U64, P, P, P]
        L.ld_logdet_cheb_noalloc.argtypes = [P, D, D, I, I, U64, P, P, P]
        L.ld_logabsdet_cheb.argtypes = [P, P, D, D, I, I, U64, P, P, P]
        L.ld_logdet_cheb_grad.argtypes = [P, D, D, I, I, U64, D, P, I, P, P, P]
        L.ld_logdet_cheb_batched.argtypes = [I, P, P, P, P, I, U64, P, P, P]
        L.ld_gershgorin.argtypes = [P, P, P, P]
        L.ld_gershgorin_batched.argtypes = [I, P, P, P, P]
        L.ld_probes.argtypes = [U64, I, I64, P, P]
        L.ld_transpose.argtypes = [P, P, P, P, P]
        L.ld_workspace_bytes.argtypes = [P, I, I, I, I]
        L.ld_workspace_bytes.restype = SZ
        L.ld_copy.argtypes = [P, P, SZ, P, P]
        L.ld_spectral_estimate.argtypes = [P, P, I, I, U64, P, P, P]
        L.ld_spectral_estimate.restype = I
        L.ld_laplacian_minor.argtypes = [P, I64, P, P, P, ctypes.c_int32, P, P]
        L.ld_logdet_taylor.argtypes = [P, D, D, I, I, U64, P, P, P]
        L.ld_quadratic_form.argtypes = [P, P, P, P]
        L.ld_log_spanning_trees.argtypes = [P, I64, I, I, U64, I, P, P, P]
        L.ld_clear_cache.argtypes = []
        L.ld_last_error.restype = ctypes.c_char_p
        L.ld_version.restype = ctypes.c_char_p
        for f in ("ld_logdet_cheb", "ld_logdet_cheb_noalloc", "ld_logabsdet_cheb", "ld_logdet_cheb_grad", "ld_logdet_cheb_batched",
                  "ld_gershgorin", "ld_probes", "ld_transpose", "ld_copy", "ld_clear_cache", "ld_laplacian_minor",
                  "ld_log_spanning_trees", "ld_logdet_taylor", "ld_quadratic_form", "ld_gershgorin_batched"):
            getattr(L, f).restype = I
        _lib = L
    return _lib


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise LogdetChebError(f"{what} failed ({rc}): {lib().ld_last_error().decode()}")
    return rc


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


@dataclass
class DeviceCSR:
    """Square CSR matrix whose arrays live on a GPU: row_ptr int64, col int32, values f64/f32/bf16.

    The effective matrix is values + diag_shift * I (the shift stays an FP64 scalar)."""

    row_ptr: torch.Tensor
    col: torch.Tensor
    values: torch.Tensor
    diag_shift: float = 0.0
    _c: _CSR = field(default=None, repr=False)

    @property
    def d(self) -> int:
        return int(self.row_ptr.shape[0]) - 1

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @classmethod
    def from_host(cls, B, device="cuda", dtype: torch.dtype | None = None, diag_shift: float = 0.0) -> "DeviceCSR":
        """From any object with numpy ``row_ptr``, ``col``, ``val`` (float64) and ``storage``."""
        if dtype is None:
            dtype = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[getattr(B, "storage", "f64")]
        rp = torch.as_tensor(B.row_ptr, dtype=torch.int64).to(device)
        col = torch.as_tensor(B.col, dtype=torch.int32).to(device)
        val = torch.as_tensor(B.val, dtype=torch.float64).to(dtype).to(device)
        return cls(rp, col, val, float(diag_shift))

    def c(self) -> _CSR:
        for t, dt in ((self.row_ptr, torch.int64), (self.col, torch.int32)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise LogdetChebError("row_ptr/col must be contiguous int64/int32 device tensors")
        if self.values.dtype not in _DTYPE or not self.values.is_cuda or not self.values.is_contiguous():
            raise LogdetChebError("values must be a contiguous float64/float32/bfloat16 device tensor")
        d = self.d
        return _CSR(d, d, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(), self.values.data_ptr(),
                    _DTYPE[self.values.dtype], 0, float(self.diag_shift))


def _opts(vec_f64=None, tile=0, timing=False, workspace=None, ckpt_stride=0, moments=None, probes=None,
          probe_tile=0, plain=False):
    o = _Opts()
    o.plain_recurrence = 1 if plain else 0
    o.vec_f64 = 0 if vec_f64 is None else (1 if vec_f64 else 2)
    o.tile = int(tile)
    o.probe_tile = int(probe_tile)
    o.timing = 1 if timing else 0
    o.ckpt_stride = int(ckpt_stride)
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    if moments is not None:
        o.moments_out = moments.ctypes.data
    if probes is not None:
        o.probe_out = probes.ctypes.data
    return o


def _result(r: _Result, rc: int) -> dict:
    return {"logdet": r.logdet, "std_err": r.std_err, "poly_bound": r.poly_bound, "grad_shift": r.grad_shift,
            "kernel_ms": r.kernel_ms, "kernel_launches": r.kernel_launches, "adjoint_ms": r.adjoint_ms,
            "adjoint_launches": r.adjoint_launches, "n": r.n, "M": r.M,
            "flags": r.flags, "adjoint_form": _ADJ_FORMS.get(r.adjoint_form), "plane_tiles": r.plane_tiles,
            "staged_steps": r.staged_steps, "status": rc}


def ld_logdet_cheb(B: DeviceCSR, a: float, b: float, n: int, M: int, seed: int, *, vec_f64=None, tile=0,
                   probe_tile=0, timing=False, workspace=None, want_moments=False, want_probes=False,
                   plain=False, stream=None) -> dict:
    """Algorithm 1 in [a, b] form: estimate of log det(B + diag_shift I)."""
    import numpy as np

    mom = np.zeros((M, n + 1)) if want_moments else None
    pv = np.zeros(M) if want_probes else None
    o = _opts(vec_f64, tile, timing, workspace, moments=mom, probes=pv, probe_tile=probe_tile, plain=plain)
    r = _Result()
    cb = B.c()
    rc = _check(lib().ld_logdet_cheb(ctypes.byref(cb), float(a), float(b), int(n), int(M), int(seed) & (2**64 - 1),
                                     ctypes.byref(o), _stream_ptr(stream), ctypes.byref(r)), "ld_logdet_cheb")
    out = _result(r, rc)
    if mom is not None:
        out["moments"] = mom
    if pv is not None:
        out["s"] = pv
    return out


def ld_logdet_cheb_noalloc(B: DeviceCSR, a: float, b: float, n: int, M: int, seed: int, *, vec_f64=None, tile=0,
                           probe_tile=0, want_moments=False, want_probes=False, plain=False, stream=None) -> dict:
    """ld_logdet_cheb on the library's fixed scratch array: no device allocation (64 MiB limit)."""
    import numpy as np

    mom = np.zeros((M, n + 1)) if want_moments else None
    pv = np.zeros(M) if want_probes else None
    o = _opts(vec_f64, tile, False, None, moments=mom, probes=pv, probe_tile=probe_tile, plain=plain)
    r = _Result()
    cb = B.c()
    rc = _check(lib().ld_logdet_cheb_noalloc(ctypes.byref(cb), float(a), float(b), int(n), int(M),
                                             int(seed) & (2**64 - 1), ctypes.byref(o), _stream_ptr(stream),
                                             ctypes.byref(r)), "ld_logdet_cheb_noalloc")
    out = _result(r, rc)
    if mom is not None:
        out["moments"] = mom
    if pv is not None:
        out["s"] = pv
    return out


def ld_logabsdet_cheb(C: DeviceCSR, Ct: DeviceCSR | None, smin: float, smax: float, n: int, M: int, seed: int, *,
                      vec_f64=None, tile=0, timing=False, workspace=None, want_probes=False, plain=False,
                      stream=None) -> dict:
    """Algorithm 2: estimate of log|det C| = (1/2) log det(C^T C)."""
    import numpy as np

    pv = np.zeros(M) if want_probes else None
    o = _opts(vec_f64, tile, timing, workspace, probes=pv, plain=plain)
    r = _Result()
    cc = C.c()
    ct = Ct.c() if Ct is not None else None
    rc = _check(lib().ld_logabsdet_cheb(ctypes.byref(cc), ctypes.byref(ct) if ct is not None else None, float(smin),
                                        float(smax), int(n), int(M), int(seed) & (2**64 - 1), ctypes.byref(o),
                                        _stream_ptr(stream), ctypes.byref(r)), "ld_logabsdet_cheb")
    out = _result(r, rc)
    if pv is not None:
        out["s"] = pv
    return out


def ld_logdet_taylor(B: DeviceCSR, a: float, b: float, n: int, M: int, seed: int, *, vec_f64=None, tile=0,
                     timing=False, workspace=None, want_moments=False, want_probes=False, stream=None) -> dict:
    """Taylor-series comparator (Section 5.1): d log(a+b) - sum_{k<=n} tr(A^k)/k by the probes,
    A = I - (B + diag_shift I)/(a + b)."""
    import numpy as np

    mom = np.zeros((M, n + 1)) if want_moments else None
    pv = np.zeros(M) if want_probes else None
    o = _opts(vec_f64, tile, timing, workspace, moments=mom, probes=pv)
    r = _Result()
    cb = B.c()
    rc = _check(lib().ld_logdet_taylor(ctypes.byref(cb), float(a), float(b), int(n), int(M), int(seed) & (2**64 - 1),
                                       ctypes.byref(o), _stream_ptr(stream), ctypes.byref(r)), "ld_logdet_taylor")
    out = _result(r, rc)
    if mom is not None:
        out["moments"] = mom
    if pv is not None:
        out["s"] = pv
    return out


def ld_quadratic_form(B: DeviceCSR, x: torch.Tensor, stream=None) -> float:
    """x^T (B + diag_shift I) x in FP64; x is a contiguous float64 device vector of length d."""
    if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != B.d:
        raise LogdetChebError("x must be a contiguous float64 device vector of length d")
    out = ctypes.c_double(0.0)
    cb = B.c()
    _check(lib().ld_quadratic_form(ctypes.byref(cb), x.data_ptr(), _stream_ptr(stream), ctypes.byref(out)),
           "ld_quadratic_form")
    return out.value


def ld_laplacian_minor(adj: DeviceCSR, hub: int, dtype: torch.dtype = torch.float32, stream=None) -> tuple:
    """Laplacian of a graph (adjacency pattern ``adj``) with the hub's row and column removed.
    Returns (DeviceCSR of the minor, Delta_max)."""
    if dtype not in (torch.float64, torch.float32):
        raise LogdetChebError("minor values must be float64 or float32")
    m = adj.d - 1
    if m < 1:
        raise LogdetChebError("a graph needs at least 2 vertices")
    nnz = adj.nnz - m
    if nnz < m:
        raise LogdetChebError("adjacency has too few entries for a hub adjacent to every vertex")
    dev = adj.row_ptr.device
    rp = torch.empty(m + 1, dtype=torch.int64, device=dev)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    val = torch.empty(nnz, dtype=dtype, device=dev)
    dmax = ctypes.c_int64(0)
    ca = adj.c()
    _check(lib().ld_laplacian_minor(ctypes.byref(ca), int(hub), rp.data_ptr(), col.data_ptr(), val.data_ptr(),
                                    _DTYPE[dtype], ctypes.byref(dmax), _stream_ptr(stream)), "ld_laplacian_minor")
    return DeviceCSR(rp, col, val), int(dmax.value)


def ld_log_spanning_trees(adj: DeviceCSR, hub: int, n: int, M: int, seed: int, *, method: int = 1, vec_f64=None,
                          tile=0, timing=False, workspace=None, want_probes=False, plain=False, stream=None) -> dict:
    """Estimate of log tau(G) for a graph whose vertex ``hub`` is adjacent to every other vertex:
    method 1 = Algorithm 2 on L(hub) (the spanning-tree corollary), method 0 = Algorithm 1."""
    import numpy as np

    pv = np.zeros(M) if want_probes else None
    o = _opts(vec_f64, tile, timing, workspace, probes=pv, plain=plain)
    r = _Result()
    ca = adj.c()
    rc = _check(lib().ld_log_spanning_trees(ctypes.byref(ca), int(hub), int(n), int(M), int(seed) & (2**64 - 1),
                                            int(method), ctypes.byref(o), _stream_ptr(stream), ctypes.byref(r)),
                "ld_log_spanning_trees")
    out = _result(r, rc)
    if pv is not None:
        out["s"] = pv
    return out


def ld_logdet_cheb_grad(B: DeviceCSR, a: float, b: float, n: int, M: int, seed: int, grad_output: float = 1.0, *,
                        grad_dtype: torch.dtype | None = None, vec_f64=None, ckpt_stride=0, tile=0, timing=False,
                        workspace=None, plain=False, stream=None) -> tuple:
    """Gradient of the Algorithm 1 estimate w.r.t. the stored entries of B (a, b fixed).

    For a symmetric pattern the value per stored entry is the derivative along symmetric
    perturbations, (dGamma/dB_ij + dGamma/dB_ji)/2.  Returns (result dict with 'logdet' and
    'grad_shift', grad tensor of length nnz)."""
    if grad_dtype is None:
        grad_dtype = torch.float64 if B.values.dtype == torch.float64 else torch.float32
    if grad_dtype not in (torch.float64, torch.float32):
        raise LogdetChebError("grad_dtype must be float64 or float32")
    grad = torch.empty(B.nnz, dtype=grad_dtype, device=B.values.device)
    o = _opts(vec_f64, tile, timing, workspace, ckpt_stride=ckpt_stride, plain=plain)
    r = _Result()
    cb = B.c()
    rc = _check(lib().ld_logdet_cheb_grad(ctypes.byref(cb), float(a), float(b), int(n), int(M),
                                          int(seed) & (2**64 - 1), float(grad_output), grad.data_ptr(),
                                          _DTYPE[grad_dtype], ctypes.byref(o), _stream_ptr(stream), ctypes.byref(r)),
                "ld_logdet_cheb_grad")
    return _result(r, rc), grad


def ld_logdet_cheb_batched(mats: list, a, b, n, M: int, seed: int, *, vec_f64=None, tile=0, timing=False,
                           plain=False, stream=None) -> list:
    """Batched Algorithm 1: matrix i uses [a[i], b[i]], degree n[i] and probe seed seed + i.
    With a = b = None every member gets its Gershgorin interval, computed in one device pass."""
    count = len(mats)
    if (a is None) != (b is None):
        raise LogdetChebError("give both a and b, or neither")
    arr = (_CSR * count)(*[m.c() for m in mats])
    av = (ctypes.c_double * count)(*[float(x) for x in a]) if a is not None else None
    bv = (ctypes.c_double * count)(*[float(x) for x in b]) if b is not None else None
    nv = (ctypes.c_int * count)(*[int(x) for x in n])
    res = (_Result * count)()
    o = _opts(vec_f64, tile, timing, plain=plain)
    rc = _check(lib().ld_logdet_cheb_batched(count, arr, av, bv, nv, int(M), int(seed) & (2**64 - 1),
                                             ctypes.byref(o), _stream_ptr(stream), res), "ld_logdet_cheb_batched")
    return [_result(res[i], rc) for i in range(count)]


def ld_gershgorin_batched(mats: list, stream=None) -> tuple:
    """Gershgorin intervals of every matrix of a batch in one device pass: (list of a, list of b)."""
    count = len(mats)
    arr = (_CSR * count)(*[m.c() for m in mats])
    av = (ctypes.c_double * count)()
    bv = (ctypes.c_double * count)()
    _check(lib().ld_gershgorin_batched(count, arr, av, bv, _stream_ptr(stream)), "ld_gershgorin_batched")
    return list(av), list(bv)


def ld_gershgorin(B: DeviceCSR, stream=None) -> tuple:
    """Gershgorin interval of B + diag_shift I, computed on the device in FP64."""
    a = ctypes.c_double()
    b = ctypes.c_double()
    cb = B.c()
    _check(lib().ld_gershgorin(ctypes.byref(cb), ctypes.byref(a), ctypes.byref(b), _stream_ptr(stream)),
           "ld_gershgorin")
    return a.value, b.value


def ld_spectral_estimate(B: DeviceCSR, iters: int = 200, gram: bool = False, Ct: DeviceCSR | None = None,
                         seed: int = 0, stream=None) -> tuple:
    """Extreme Ritz values of B + diag_shift I (or of C^T C with gram=True) after `iters` Lanczos
    steps in FP64: estimates from inside the spectrum, not bounds."""
    lo = ctypes.c_double()
    hi = ctypes.c_double()
    cb = B.c()
    ct = Ct.c() if Ct is not None else None
    _check(lib().ld_spectral_estimate(ctypes.byref(cb), ctypes.byref(ct) if ct is not None else None,
                                      1 if gram else 0, int(iters), int(seed) & (2**64 - 1), _stream_ptr(stream),
                                      ctypes.byref(lo), ctypes.byref(hi)), "ld_spectral_estimate")
    return lo.value, hi.value


def ld_probes(seed: int, M: int, rows: int, device="cuda", stream=None) -> torch.Tensor:
    """The probe block as an int8 (rows, M) device tensor of +1/-1."""
    out = torch.empty((rows, M), dtype=torch.int8, device=device)
    _check(lib().ld_probes(int(seed) & (2**64 - 1), int(M), int(rows), out.data_ptr(), _stream_ptr(stream)),
           "ld_probes")
    return out


def ld_transpose(C: DeviceCSR, stream=None) -> DeviceCSR:
    """C^T in CSR form (rows sorted by column), built on the device."""
    rp = torch.empty(C.d + 1, dtype=torch.int64, device=C.values.device)
    col = torch.empty(C.nnz, dtype=torch.int32, device=C.values.device)
    val = torch.empty(C.nnz, dtype=C.values.dtype, device=C.values.device)
    cc = C.c()
    _check(lib().ld_transpose(ctypes.byref(cc), rp.data_ptr(), col.data_ptr(), val.data_ptr(), _stream_ptr(stream)),
           "ld_transpose")
    return DeviceCSR(rp, col, val, C.diag_shift)


def ld_workspace_bytes(B: DeviceCSR, n: int, M: int, mode: int = 0, vec_f64: bool | None = None) -> int:
    cb = B.c()
    v = (B.values.dtype == torch.float64) if vec_f64 is None else bool(vec_f64)
    return int(lib().ld_workspace_bytes(ctypes.byref(cb), int(n), int(M), int(mode), 1 if v else 0))


def ld_copy(dst: torch.Tensor, src: torch.Tensor, stream=None) -> float:
    """Copy src into dst with the library's streaming kernel; returns the kernel time in ms."""
    nbytes = min(dst.numel() * dst.element_size(), src.numel() * src.element_size())
    ms = ctypes.c_double()
    _check(lib().ld_copy(dst.data_ptr(), src.data_ptr(), nbytes, _stream_ptr(stream), ctypes.byref(ms)), "ld_copy")
    return ms.value


def ld_clear_cache() -> None:
    """Release the library's cached batched graphs and autotuning results."""
    _check(lib().ld_clear_cache(), "ld_clear_cache")


def ld_version() -> str:
    return lib().ld_version().decode()


class LogdetCheb(torch.autograd.Function):
    """log det(B + shift I) estimate with a gradient on B's sparsity pattern.

    forward(values, shift, row_ptr, col, a, b, n, M, seed) -> scalar float64 tensor.
    The gradient flows to ``values`` (one entry per stored element) and to ``shift`` (a 0-d
    tensor); a and b are treated as constants.  The backward pass runs the library's adjoint
    kernels with checkpointed recomputation of the forward recurrence."""

    @staticmethod
    def forward(ctx, values, shift, row_ptr, col, a, b, n, M, seed):
        B = DeviceCSR(row_ptr, col, values.detach().contiguous(), float(shift))
        r = ld_logdet_cheb(B, a, b, n, M, seed)
        ctx.save_for_backward(values, row_ptr, col)
        ctx.cfg = (float(shift), a, b, n, M, seed)
        ctx.std_err = r["std_err"]  # read back through the output's grad_fn by ``logdet``
        return torch.tensor(r["logdet"], dtype=torch.float64, device=values.device)

    @staticmethod
    def backward(ctx, g):
        values, row_ptr, col = ctx.saved_tensors
        shift, a, b, n, M, seed = ctx.cfg
        B = DeviceCSR(row_ptr, col, values.detach().contiguous(), shift)
        gdt = torch.float64 if values.dtype == torch.float64 else torch.float32
        r, grad = ld_logdet_cheb_grad(B, a, b, n, M, seed, float(g.item()), grad_dtype=gdt)
        gshift = torch.tensor(r["grad_shift"], dtype=torch.float64, device=values.device)
        return grad.to(values.dtype), gshift, None, None, None, None, None, None, None


def as_device_csr(B, diag_shift: float = 0.0) -> DeviceCSR:
    """A DeviceCSR as it is, or a square torch sparse CSR tensor on the GPU viewed as one (row
    pointers as int64 and columns as int32, copied only if their dtype differs)."""
    if isinstance(B, DeviceCSR):
        return B
    if torch.is_tensor(B) and B.layout == torch.sparse_csr:
        if B.dim() != 2 or B.shape[0] != B.shape[1]:
            raise LogdetChebError("the sparse CSR tensor must be square")
        return DeviceCSR(B.crow_indices().to(torch.int64).contiguous(), B.col_indices().to(torch.int32).contiguous(),
                         B.values().contiguous(), float(diag_shift))
    raise LogdetChebError("expected a DeviceCSR or a torch sparse CSR tensor")


def logdet(B, n: int, M: int, seed: int = 0, a: float | None = None, b: float | None = None,
           shift: float = 0.0) -> tuple:
    """Algorithm 1 on a DeviceCSR or a square torch sparse CSR tensor (plus shift * I): returns
    (estimate as a float64 0-d tensor, standard error).  When the stored values require grad the
    estimate carries the gradient with respect to them (the library's adjoint, a and b held
    fixed); the bounds default to the Gershgorin interval."""
    D = as_device_csr(B, shift)
    if a is None or b is None:
        ga, gb = ld_gershgorin(D)
        a = ga if a is None else a
        b = gb if b is None else b
        if not a > 0:
            raise LogdetChebError(f"Gershgorin lower bound {a} is not positive; pass a > 0 explicitly")
    vals = B.values() if torch.is_tensor(B) else D.values
    if vals.requires_grad:
        st = torch.tensor(float(shift), dtype=torch.float64, device=vals.device)
        out = LogdetCheb.apply(vals, st, D.row_ptr, D.col, float(a), float(b), int(n), int(M), int(seed))
        return out, out.grad_fn.std_err
    r = ld_logdet_cheb(D, a, b, n, M, seed)
    return torch.tensor(r["logdet"], dtype=torch.float64, device=vals.device), r["std_err"]


def logdet_cheb(B: DeviceCSR, n: int, M: int, seed: int = 0, a: float | None = None, b: float | None = None,
                **kw) -> dict:
    """Estimate log det(B + diag_shift I); bounds default to the Gershgorin interval (device)."""
    if a is None or b is None:
        ga, gb = ld_gershgorin(B)
        a = ga if a is None else a
        b = gb if b is None else b
        if not a > 0:
            raise LogdetChebError(f"Gershgorin lower bound {a} is not positive; pass a > 0 explicitly")
    return ld_logdet_cheb(B, a, b, n, M, seed, **kw)

"""Maximum-likelihood estimation of a Gaussian Markov random field's coupling with the stochastic
Chebyshev log-determinant (the GMRF experiment of Section 5.2).

The field has precision J(rho) = I - rho A on a graph with adjacency A: J_ii = 1 and J_ij = -rho
on every edge, so rho is the partial correlation of neighbours.  For a sample x the
log-likelihood is, up to a constant,

    l(rho) = (1/2) log det J(rho) - (1/2) x^T J(rho) x,

with the log-determinant from Algorithm 1 (or Algorithm 2, as in the paper's experiment) and the
quadratic term from the library's FP64 quadratic form.  Gershgorin gives the spectral interval
[1 - |rho| D, 1 + |rho| D] (D the largest number of neighbours), which is what the estimator is
given.  The derivative dl/drho comes from the library's adjoint (the gradient with respect to
J's stored entries) through torch's chain rule.
"""
from __future__ import annotations

import torch

from . import (DeviceCSR, LogdetCheb, LogdetChebError, ld_logabsdet_cheb, ld_logdet_cheb,
               ld_quadratic_form)


class GMRF:
    """GMRF with precision J(rho) = I - rho A on the graph whose CSR pattern (diagonal entries
    included, int64 row pointers and int32 columns on the device) is given."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, dtype: torch.dtype = torch.float32):
        if dtype not in (torch.float32, torch.float64):
            raise LogdetChebError("values must be float32 or float64")
        self.row_ptr = row_ptr
        self.col = col
        self.dtype = dtype
        d = row_ptr.numel() - 1
        counts = row_ptr[1:] - row_ptr[:-1]
        rows = torch.repeat_interleave(torch.arange(d, device=row_ptr.device), counts)
        self.is_diag = col.to(torch.int64) == rows
        if int(self.is_diag.sum()) != d:
            raise LogdetChebError("the pattern must store every diagonal entry")
        self.max_neighbours = int((counts - 1).max()) if d > 0 else 0
        self.adjacency = DeviceCSR(row_ptr, col, (~self.is_diag).to(torch.float64))

    @property
    def d(self) -> int:
        return self.row_ptr.numel() - 1

    def values(self, rho) -> torch.Tensor:
        """Stored entries of J(rho): 1 on the diagonal, -rho elsewhere (rounded to the value type)."""
        if not torch.is_tensor(rho):
            rho = torch.tensor(float(rho), dtype=torch.float64, device=self.row_ptr.device)
        one = torch.ones((), dtype=torch.float64, device=self.row_ptr.device)
        return torch.where(self.is_diag, one, -rho).to(self.dtype)

    def precision(self, rho: float) -> DeviceCSR:
        return DeviceCSR(self.row_ptr, self.col, self.values(rho).contiguous())

    def bounds(self, rho: float) -> tuple:
        """Gershgorin interval of J(rho)."""
        r = abs(float(rho)) * self.max_neighbours
        if not r < 1.0:
            raise LogdetChebError(f"J(rho) is not diagonally dominant for rho={rho}")
        return 1.0 - r, 1.0 + r

    def loglik(self, rho: float, x: torch.Tensor, n: int, M: int, seed: int, method: int = 1) -> dict:
        """(1/2) log det J(rho) - (1/2) x^T J(rho) x, with the log det from Algorithm 1
        (method 1) or Algorithm 2 with C = J(rho) (method 2)."""
        a, b = self.bounds(rho)
        J = self.precision(rho)
        if method == 1:
            r = ld_logdet_cheb(J, a, b, n, M, seed)
        elif method == 2:
            r = ld_logabsdet_cheb(J, J, a, b, n, M, seed)  # J is its own transpose
        else:
            raise LogdetChebError("method must be 1 or 2")
        q = ld_quadratic_form(J, x)
        return {"rho": float(rho), "logdet": r["logdet"], "std_err": r["std_err"], "quad": q,
                "loglik": 0.5 * r["logdet"] - 0.5 * q}

    def sweep(self, rhos, x: torch.Tensor, n: int, M: int, seed: int, method: int = 1) -> list:
        """l(rho) for every rho given, with the same probes at each value."""
        return [self.loglik(r, x, n, M, seed, method) for r in rhos]

    def loglik_grad(self, rho: float, x: torch.Tensor, n: int, M: int, seed: int) -> tuple:
        """(l(rho), dl/drho): the log det's derivative runs through the library's adjoint."""
        a, b = self.bounds(rho)
        rt = torch.tensor(float(rho), dtype=torch.float64, device=self.row_ptr.device, requires_grad=True)
        vals = self.values(rt)
        shift = torch.zeros((), dtype=torch.float64, device=self.row_ptr.device)
        gamma = LogdetCheb.apply(vals, shift, self.row_ptr, self.col, a, b, n, M, seed)
        gamma.backward()
        dgamma = float(rt.grad)
        q = ld_quadratic_form(self.precision(rho), x)
        xax = ld_quadratic_form(self.adjacency, x)  # d(x^T J x)/drho = -x^T A x
        return 0.5 * float(gamma.detach()) - 0.5 * q, 0.5 * dgamma + 0.5 * xax

    def fit(self, x: torch.Tensor, rho0: float, n: int, M: int, seed: int, step: float = 0.02, iters: int = 40,
            tol: float = 1e-7) -> dict:
        """Maximum-likelihood rho.  l is concave in rho (its second derivative is
        -(1/2) sum_i lambda_i^2 / (1 - rho lambda_i)^2 for the eigenvalues lambda_i of A), so dl/drho
        decreases: bracket its root by steps of doubling length from rho0 inside the diagonally
        dominant range, then refine by regula falsi with the Illinois modification."""
        lim = 0.999 / max(self.max_neighbours, 1)
        path = []

        def grad(r):
            _, gr = self.loglik_grad(r, x, n, M, seed)
            path.append((r, gr))
            return gr

        def clamp(r):
            return min(max(r, -lim), lim)

        a = clamp(float(rho0))
        ga = grad(a)
        if ga == 0.0:
            return {"rho": a, "dloglik": ga, "path": path}
        s = -step if ga < 0 else step
        while True:
            b = clamp(a + s)
            gb = grad(b)
            if (gb < 0) != (ga < 0):
                break
            if abs(b) >= lim:
                raise LogdetChebError("dl/drho does not change sign inside the admissible range")
            a, ga, s = b, gb, 2 * s
        c, gc, side = b, gb, 0
        for _ in range(iters):
            c = b - gb * (b - a) / (gb - ga)
            gc = grad(c)
            if abs(gc) <= tol * self.d or abs(b - a) < 1e-12:
                break
            if (gc < 0) == (gb < 0):
                b, gb = c, gc
                if side == -1:
                    ga *= 0.5
                side = -1
            else:
                a, ga = c, gc
                if side == 1:
                    gb *= 0.5
                side = 1
        return {"rho": c, "dloglik": gc, "path": path}

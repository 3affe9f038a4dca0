"""Differentiable solve of -div(exp(theta) grad u) + b u = f (eq. (1.1), FD of Sec. 3.1 / 3.2)
with the RHIF-preconditioned CG of the library.

The forward pass assembles A(exp theta) on the device, factors it and solves A u = f. The
backward pass reuses that factorization for the adjoint solve A lam = dL/du (A is symmetric)
and forms dL/dtheta per cell with the library's gradient kernel (rhif_grad_log_a); dL/df is
lam. Everything runs through the C ABI; this module only marshals tensors.
"""
from __future__ import annotations

import torch

from . import rhif


class _SolveLogA(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, f, dim, n, b, leaf, eps, rtol, maxit):
        N = n ** dim
        rhif._need((theta.detach().reshape(-1), "theta", (n + 1) ** dim), (f.detach().reshape(-1), "f", N),
                   *([(b.detach().reshape(-1), "b", N)] if b is not None else []))
        a = torch.exp(theta.detach()).contiguous()
        csr = rhif.assemble_fd(dim, n, a.reshape(-1), None if b is None else b.detach().reshape(-1))
        F = rhif.Factor(dim, n, csr, leaf, eps, 1)
        u, it, rr = F.pcg(f.detach().reshape(-1).contiguous(), rtol, maxit)
        # the factor is kept for the adjoint solve of the (single) backward pass and released
        # there; it is released with the graph if no backward pass runs
        ctx.F = F
        ctx.dims = (dim, n, rtol, maxit, f.shape, None if b is None else b.shape)
        ctx.iters = it
        ctx.save_for_backward(a, u)
        return u

    @staticmethod
    def backward(ctx, gu):
        F = ctx.F
        if F is None:
            raise RuntimeError("solve_log_a: the factorization was released after the first backward pass; "
                               "a second backward pass (retain_graph=True) needs a new forward solve")
        a, u = ctx.saved_tensors
        dim, n, rtol, maxit, fshape, bshape = ctx.dims
        try:
            lam, it, rr = F.pcg(gu.reshape(-1).contiguous(), rtol, maxit)
        finally:
            F.close()
            ctx.F = None
        g = rhif.grad_log_a(dim, n, a.reshape(-1), u, lam).reshape(a.shape)
        # A = h^-2 K(a) + diag(b): dL/db_i = -lam_i u_i
        gb = (-(lam * u)).reshape(bshape) if bshape is not None and ctx.needs_input_grad[4] else None
        return g, lam.reshape(fshape), None, None, gb, None, None, None, None


def solve_log_a(theta: torch.Tensor, f: torch.Tensor, dim: int, n: int, b: torch.Tensor | None = None,
                leaf: int = 16, eps: float = 1e-6, rtol: float = 1e-12, maxit: int = 500) -> torch.Tensor:
    """u with A(exp theta) u = f, differentiable with respect to theta ((n+1)^dim cell values,
    c_1 fastest), f (N values) and the reaction term b (N values or None). theta, f and b are
    float64 device tensors. One backward pass per forward solve: the factorization is
    released after it."""
    return _SolveLogA.apply(theta, f, dim, n, b, leaf, eps, rtol, maxit)

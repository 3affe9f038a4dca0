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
        a = torch.exp(theta.detach()).contiguous()
        csr = rhif.assemble_fd(dim, n, a.reshape(-1), b)
        F = rhif.Factor(dim, n, csr, leaf, eps, 1)
        u, it, rr = F.pcg(f.detach().reshape(-1).contiguous(), rtol, maxit)
        ctx.F = F
        ctx.dims = (dim, n, rtol, maxit, f.shape)
        ctx.iters = it
        ctx.save_for_backward(a, u)
        return u

    @staticmethod
    def backward(ctx, gu):
        a, u = ctx.saved_tensors
        dim, n, rtol, maxit, fshape = ctx.dims
        F = ctx.F
        lam, it, rr = F.pcg(gu.reshape(-1).contiguous(), rtol, maxit)
        g = rhif.grad_log_a(dim, n, a.reshape(-1), u, lam).reshape(a.shape)
        F.close()
        ctx.F = None
        return g, lam.reshape(fshape), None, None, None, None, None, None, None


def solve_log_a(theta: torch.Tensor, f: torch.Tensor, dim: int, n: int, b: torch.Tensor | None = None,
                leaf: int = 16, eps: float = 1e-6, rtol: float = 1e-12, maxit: int = 500) -> torch.Tensor:
    """u with A(exp theta) u = f, differentiable with respect to theta ((n+1)^dim cell values,
    c_1 fastest) and f (N values). theta, f and b are float64 device tensors."""
    return _SolveLogA.apply(theta, f, dim, n, b, leaf, eps, rtol, maxit)

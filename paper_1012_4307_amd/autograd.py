"""Differentiable ECS Helmholtz solve: u = A(k^2)^{-1} f with A = -Lap - diag(k^2)
on the ECS grid, as a torch.autograd.Function.

Backward (adjoint method).  PyTorch hands backward the gradient
g = dL/dRe(u) + i dL/dIm(u) of a real loss.  Since dA/dk^2_c = -e_c e_c^T,
  dL/dk^2_c = Re(lam_c u_c),   dL/df = conj(lam),   where A^T lam = conj(g)
(plain transpose, solved by the library's adjoint solve with the same
multigrid preconditioner).  k^2 lives on the nodes, so the gradient is one
real number per node; boundary nodes get zero.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import Krylov, Solver


class HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k2: torch.Tensor, f: torch.Tensor, solver: Solver, krylov: Optional[Krylov],
                adjoint_krylov: Optional[Krylov]):
        if k2.data_ptr() != solver.k2.data_ptr() or not torch.equal(k2, solver.k2):
            solver.reset_k2(k2.detach().contiguous())
        u, st = solver.solve(f.detach().contiguous(), krylov=krylov)
        if st["status"] != 0:
            raise RuntimeError(f"forward solve did not converge: {st}")
        ctx.solver = solver
        ctx.k2_dtype = k2.dtype
        ctx.adjoint_krylov = adjoint_krylov or krylov
        ctx.save_for_backward(u)
        ctx.stats = st
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        S = ctx.solver
        lam, st = S.solve_adjoint(torch.conj(grad_u).resolve_conj().contiguous(), krylov=ctx.adjoint_krylov)
        if st["status"] != 0:
            raise RuntimeError(f"adjoint solve did not converge: {st}")
        # the gradient is formed in FP64 and returned in k2's own dtype
        grad_k2 = S.grad_k2(lam, u).to(ctx.k2_dtype) if ctx.needs_input_grad[0] else None
        grad_f = torch.conj(lam).resolve_conj() if ctx.needs_input_grad[1] else None
        return grad_k2, grad_f, None, None, None


def helmholtz_solve(solver: Solver, k2: torch.Tensor, f: torch.Tensor, krylov: Optional[Krylov] = None,
                    adjoint_krylov: Optional[Krylov] = None) -> torch.Tensor:
    """u = A(k2)^{-1} f on the solver's grid, differentiable in k2 (float64 or
    float32) and f (complex128).  The solver is re-pointed at k2 when it changes."""
    return HelmholtzSolve.apply(k2, f, solver, krylov, adjoint_krylov)

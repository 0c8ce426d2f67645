"""Differentiable solve: x = A(k)^{-1} b as a torch.autograd.Function.

Forward: one sem_pcg_solve.  Backward for a cotangent xbar of the
copy-consistent solution x_L:
  adjoint right-hand side  Q^T xbar   (sum over the copies of each node),
  adjoint solve            A(k) lam = Q^T xbar       (A is symmetric: same solve),
  kbar_q = -sum_ab (D_a lam_L)_q G_ab,q (D_b x_L)_q   (sem_ax_backward),
  bbar   = lam_L / multiplicity  (the solve reads b as the mean of its copies).
"""

from __future__ import annotations

import torch

from . import api


class SemSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k, b, mesh, h2, rtol, max_iter):
        with torch.no_grad():
            x, stats = api.solve(mesh, b.detach().contiguous(),
                                 k=None if k is None else k.detach().contiguous(),
                                 h2=h2, rtol=rtol, max_iter=max_iter)
        ctx.mesh, ctx.h2, ctx.rtol, ctx.max_iter = mesh, h2, rtol, max_iter
        ctx.stats = stats
        ctx.has_k = k is not None
        ctx.save_for_backward(k if k is not None else torch.empty(0, device=b.device), x)
        return x

    @staticmethod
    def backward(ctx, xbar):
        k, x = ctx.saved_tensors
        k = k if ctx.has_k else None
        mesh = ctx.mesh
        with torch.no_grad():
            rhs = api.gs(mesh, xbar.detach().contiguous().clone())
            lam, _ = api.solve(mesh, rhs, k=k, h2=ctx.h2, rtol=ctx.rtol, max_iter=ctx.max_iter)
            kbar = None
            if ctx.has_k and ctx.needs_input_grad[0]:
                _, kb = api.ax_backward(mesh, x, lam, need_ubar=False, need_kbar=True)
                kbar = -kb
            bbar = lam / mesh.multiplicity() if ctx.needs_input_grad[1] else None
        return kbar, bbar, None, None, None, None


def sem_solve(mesh, b, k=None, h2: float = 0.0, rtol: float = 1e-12, max_iter: int = 20000):
    """Differentiable x = A(k)^{-1} b (gradients for k and b)."""
    return SemSolve.apply(k, b, mesh, float(h2), float(rtol), int(max_iter))

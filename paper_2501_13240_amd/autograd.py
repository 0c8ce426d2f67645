"""Differentiable solve: x = A(k)^{-1} b as a torch.autograd.Function.

Forward: one sem_pcg_solve.  Backward: one sem_solve_backward, which runs the
adjoint solve A(k) lam = R Q^T xbar and forms both gradients in libsem:
  dL/dk = -sum_ab (D_a lam_L) G_ab (D_b x_L)   (the k-derivative of the operator),
  dL/db = lam_L / multiplicity                  (b is read as the mean of its copies).
This module only marshals tensors.
"""

from __future__ import annotations

import torch

from . import api


class SemSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k, b, mesh, h2, rtol, max_iter, opts):
        with torch.no_grad():
            x, stats = api.solve(mesh, b.detach().contiguous(),
                                 k=None if k is None else k.detach().contiguous(),
                                 h2=h2, rtol=rtol, max_iter=max_iter, **opts)
        ctx.mesh, ctx.h2, ctx.rtol, ctx.max_iter, ctx.opts = mesh, h2, rtol, max_iter, opts
        ctx.stats = stats
        ctx.has_k = k is not None
        ctx.save_for_backward(k if k is not None else torch.empty(0, device=b.device), x)
        return x

    @staticmethod
    def backward(ctx, xbar):
        k, x = ctx.saved_tensors
        need_k = ctx.has_k and ctx.needs_input_grad[0]
        need_b = ctx.needs_input_grad[1]
        if not (need_k or need_b):
            return None, None, None, None, None, None, None
        with torch.no_grad():
            kbar, bbar, _ = api.solve_backward(
                ctx.mesh, x, xbar.detach().contiguous(), k=k if ctx.has_k else None, h2=ctx.h2,
                need_kbar=need_k, need_bbar=need_b, rtol=ctx.rtol, max_iter=ctx.max_iter,
                **ctx.opts)
        return kbar, bbar, None, None, None, None, None


def sem_solve(mesh, b, k=None, h2: float = 0.0, rtol: float = 1e-12, max_iter: int = 20000,
              **opts):
    """Differentiable x = A(k)^{-1} b (gradients for k and b).  opts: solve
    options of api.solve (mode, precond, precond_prec, cheb_order, ...), used
    by the forward solve and by the adjoint solve of the backward."""
    return SemSolve.apply(k, b, mesh, float(h2), float(rtol), int(max_iter), dict(opts))

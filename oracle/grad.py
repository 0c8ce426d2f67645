"""O13: adjoint gradient of a solve with respect to k and b.

Test infrastructure only (see the package docstring).

For A(k) x = b with A(k) = R Q^T A_L(k) Q R^T symmetric and a loss L(x):
  A lambda = dL/dx                              (adjoint solve, same operator)
  dL/db    = lambda
  dL/dk_q  = -kbar_q(wbar = (Q R^T lambda)_L, u = (Q R^T x)_L)
with kbar the backward contraction of the element operator.
"""

from __future__ import annotations

import numpy as np

from .operator import kgrad_contraction


def solve_and_adjoint_gradient(prob, b, target, rtol=1e-13, max_iter=20000):
    """L = sum over free unique nodes of (x - target)^2.

    Returns dict(x, L, lam, kbar_local (E,P), iters, adj_iters)."""
    fwd = prob.solve(b, rtol=rtol, max_iter=max_iter)
    x = fwd["x"]
    diff = x - target
    L = float(diff @ diff)
    adj = prob.solve(2.0 * diff, rtol=rtol, max_iter=max_iter)
    lam = adj["x"]
    num = prob.num
    kb = -kgrad_contraction(num.to_local(x), num.to_local(lam), prob.G, prob.N)
    return dict(x=x, L=L, lam=lam, kbar_local=kb, iters=fwd["iters"], adj_iters=adj["iters"])

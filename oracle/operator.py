"""O4/O7/a10: the element operator, its diagonal and its derivative in k.

Test infrastructure only (see the package docstring).

Weak form of -div(k grad u) + h2 u with Gauss-Lobatto quadrature on each
element, written through the reference derivatives (Sec. 2.2: tensor
contractions with (N+1)x(N+1) matrices identical for all elements, carried to
deformed elements by the chain rule):

  u_a = D_a u                              (a = r, s, t)
  v_a = k * sum_b G_ab u_b                 (pointwise)
  w   = D_r^T v_r + D_s^T v_s + D_t^T v_t + h2 B u

Backward in k (the operator is linear in k):
  kbar_q = sum_ab (D_a wbar)_q G_ab,q (D_b u)_q,
so that <wbar, A(dk) u> = sum_q dk_q kbar_q.
"""

from __future__ import annotations

import numpy as np

from .gll import deriv_matrix
from .geometry import tensor, d_r, d_s, d_t


def _dT_r(D, F):
    return np.einsum("li,ekjl->ekji", D, F)


def _dT_s(D, F):
    return np.einsum("lj,ekli->ekji", D, F)


def _dT_t(D, F):
    return np.einsum("lk,elji->ekji", D, F)


def _grads(u, N, D):
    U = tensor(u, N)
    return d_r(D, U), d_s(D, U), d_t(D, U)


def _metric_times(G, N, gr, gs, gt):
    g = [tensor(np.ascontiguousarray(G[:, c, :]), N) for c in range(6)]
    vr = g[0] * gr + g[1] * gs + g[2] * gt
    vs = g[1] * gr + g[3] * gs + g[4] * gt
    vt = g[2] * gr + g[4] * gs + g[5] * gt
    return vr, vs, vt


def local_apply(u, G, B, N, k=None, h2=0.0):
    """w = A_L u for every element; u (E, P) -> w (E, P)."""
    D = deriv_matrix(N)
    ur, us, ut = _grads(u, N, D)
    vr, vs, vt = _metric_times(G, N, ur, us, ut)
    if k is not None:
        K = tensor(k, N)
        vr, vs, vt = K * vr, K * vs, K * vt
    w = _dT_r(D, vr) + _dT_s(D, vs) + _dT_t(D, vt)
    w = w.reshape(u.shape)
    if h2 != 0.0:
        w = w + h2 * B * u
    return w


def mass_apply(u, B):
    """w = B u (diagonal mass matrix of GLL quadrature)."""
    return B * u


def local_diagonal(G, B, N, k=None, h2=0.0):
    """Diagonal of A_L at every local point (i, j, k):
      sum_l D_li^2 (kG_rr)(l,j,k) + sum_l D_lj^2 (kG_ss)(i,l,k)
    + sum_l D_lk^2 (kG_tt)(i,j,l)
    + 2 D_ii D_jj (kG_rs) + 2 D_ii D_kk (kG_rt) + 2 D_jj D_kk (kG_st)  [at (i,j,k)]
    + h2 B."""
    D = deriv_matrix(N)
    E = G.shape[0]
    kk = np.ones_like(B) if k is None else k
    g = [tensor(np.ascontiguousarray(G[:, c, :] * kk), N) for c in range(6)]
    D2 = D ** 2
    dg = np.diag(D)
    diag = (np.einsum("li,ekjl->ekji", D2, g[0])
            + np.einsum("lj,ekli->ekji", D2, g[3])
            + np.einsum("lk,elji->ekji", D2, g[5]))
    di = dg[None, None, None, :]
    dj = dg[None, None, :, None]
    dk = dg[None, :, None, None]
    diag = diag + 2.0 * (di * dj * g[1] + di * dk * g[2] + dj * dk * g[4])
    diag = diag.reshape(E, -1)
    if h2 != 0.0:
        diag = diag + h2 * B
    return diag


def kgrad_contraction(u, wbar, G, N):
    """kbar_q = sum_ab (D_a wbar)_q G_ab,q (D_b u)_q, shape (E, P)."""
    D = deriv_matrix(N)
    ur, us, ut = _grads(u, N, D)
    wr, ws, wt = _grads(wbar, N, D)
    vr, vs, vt = _metric_times(G, N, ur, us, ut)
    return (wr * vr + ws * vs + wt * vt).reshape(u.shape)

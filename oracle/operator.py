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


# --------------------------------------------------------------------------
# Low-precision contraction variant (the preconditioner's matrix-core form).
#
# The derivative contractions take 16-bit operands and accumulate exactly
# (16-bit x 16-bit products are exact in FP32; the sum is formed here in
# FP64); the pointwise metric, k and the mass term stay in working precision.
# Operands rounded: D (once), the element block of u before D_a, and each
# v_a before D_a^T.  For IEEE half precision every block is first scaled by a
# power of two that puts its largest magnitude in [2^14, 2^15), so that values
# far below one (a residual late in a solve, metric-weighted derivatives on
# small elements) keep all their bits; bfloat16 has FP32's exponent range and
# is not scaled.  Both formats round to nearest, ties to even, from FP32.

def round_to_format(x, fmt):
    """Round FP32 values of x to 'bf16' (8 significant bits, FP32 exponent
    range) or 'fp16' (IEEE binary16), nearest-even; returned as float64."""
    x32 = np.asarray(x, dtype=np.float32)
    if fmt == "fp16":
        return x32.astype(np.float16).astype(np.float64)
    if fmt != "bf16":
        raise ValueError(fmt)
    bits = x32.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def block_scale(X, fmt):
    """Per-element power-of-two scale of a block X (E, P): 2^(15 - e) with
    max|X| = f 2^e, f in [0.5, 1), for 'fp16', the exponent 15 - e limited to
    [-126, 126] so the scale and its inverse are normal FP32 numbers; 1 for
    'bf16' and zero blocks."""
    E = X.shape[0]
    if fmt != "fp16":
        return np.ones(E)
    m = np.max(np.abs(X.reshape(E, -1)), axis=1)
    _, ex = np.frexp(m)
    return np.where(m > 0, np.ldexp(1.0, np.clip(15 - ex, -126, 126)), 1.0)


def _round_block(X, fmt):
    s = block_scale(X, fmt).reshape((-1,) + (1,) * (X.ndim - 1))
    return round_to_format(X * s, fmt) / s


def local_apply_lowprec(u, G, B, N, fmt, k=None, h2=0.0):
    """w = A_L u with 16-bit contraction operands (format fmt); u (E, P)
    holding FP32 values; G, B, k in working precision."""
    D = round_to_format(deriv_matrix(N), fmt)
    U = tensor(u, N)
    Uq = _round_block(U, fmt)
    ur, us, ut = d_r(D, Uq), d_s(D, Uq), d_t(D, Uq)
    vr, vs, vt = _metric_times(G, N, ur, us, ut)
    if k is not None:
        K = tensor(k, N)
        vr, vs, vt = K * vr, K * vs, K * vt
    w = _dT_r(D, _round_block(vr, fmt)) + _dT_s(D, _round_block(vs, fmt)) \
        + _dT_t(D, _round_block(vt, fmt))
    w = w.reshape(u.shape)
    if h2 != 0.0:
        w = w + h2 * B * u
    return w


def local_apply_majorant(u, G, N, k=None):
    """|D|^T (|k| sum_b |G_ab| |D_b| |u|): the operator with every entry
    replaced by its magnitude, the scale of the rounding error bound."""
    D = np.abs(deriv_matrix(N))
    U = np.abs(tensor(u, N))
    ar, as_, at = d_r(D, U), d_s(D, U), d_t(D, U)
    vr, vs, vt = _metric_times(np.abs(G), N, ar, as_, at)
    if k is not None:
        K = np.abs(tensor(k, N))
        vr, vs, vt = K * vr, K * vs, K * vt
    return (_dT_r(D, vr) + _dT_s(D, vs) + _dT_t(D, vt)).reshape(u.shape)

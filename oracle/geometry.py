"""O3: geometric factors of the element maps (chain rule, Sec. 2.2).

Test infrastructure only (see the package docstring).

For each element the map x(r, s, t) is the degree-N interpolant of the nodal
coordinates.  With D_r = I (x) I (x) D (acting on i), D_s (on j), D_t (on k):

  J = [[x_r, x_s, x_t], [y_r, y_s, y_t], [z_r, z_s, z_t]],
  the rows of J^{-1} are grad r, grad s, grad t,
  G_ab = rho_i rho_j rho_k detJ (grad a . grad b),  a, b in {r, s, t},
  B    = rho_i rho_j rho_k detJ.

The six factors are stored in the order (rr, rs, rt, ss, st, tt) as
G[e, c, q], q the local point index (i fastest).
"""

from __future__ import annotations

import numpy as np

from .gll import gll_nodes_weights, deriv_matrix


def tensor(f: np.ndarray, N: int) -> np.ndarray:
    """(E, P) -> (E, k, j, i) view."""
    n = N + 1
    return f.reshape(f.shape[0], n, n, n)


def d_r(D, F):
    return np.einsum("il,ekjl->ekji", D, F)


def d_s(D, F):
    return np.einsum("jl,ekli->ekji", D, F)


def d_t(D, F):
    return np.einsum("kl,elji->ekji", D, F)


def jacobian(xyz: np.ndarray, N: int) -> np.ndarray:
    """J[e, q, a, b] = d x_a / d r_b."""
    D = deriv_matrix(N)
    E = xyz.shape[0]
    J = np.empty((E, (N + 1) ** 3, 3, 3))
    for a in range(3):
        X = tensor(np.ascontiguousarray(xyz[..., a]), N)
        J[:, :, a, 0] = d_r(D, X).reshape(E, -1)
        J[:, :, a, 1] = d_s(D, X).reshape(E, -1)
        J[:, :, a, 2] = d_t(D, X).reshape(E, -1)
    return J


def quadrature_weights_3d(N: int) -> np.ndarray:
    """rho_i rho_j rho_k at local point q = i + n (j + n k)."""
    _, rho = gll_nodes_weights(N)
    return np.einsum("k,j,i->kji", rho, rho, rho).reshape(-1)


def geometric_factors(xyz: np.ndarray, N: int):
    """Return (G (E,6,P), B (E,P), detJ (E,P))."""
    J = jacobian(xyz, N)
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)  # Jinv[e, q, b, a] = d r_b / d x_a
    w = quadrature_weights_3d(N)
    scale = w[None, :] * detJ
    pairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    G = np.empty((xyz.shape[0], 6, (N + 1) ** 3))
    for c, (a, b) in enumerate(pairs):
        G[:, c, :] = scale * np.sum(Jinv[:, :, a, :] * Jinv[:, :, b, :], axis=-1)
    B = scale.copy()
    return G, B, detJ

"""Convective operator of the temperature and momentum equations, with
over-integration (dealiasing).

Test infrastructure only (see the package docstring).

The Boussinesq equations of Sec. 4.1 carry the advection term u . grad T (and
u . grad u).  The paper prints no discretisation for it; the reading taken
here is the weak form on each element,

    C_e(u) T |_i = sum_q phi_i(x_q) w_q detJ_q  u(x_q) . grad T(x_q),

evaluated either on the GLL nodes themselves (collocation, aliased: the
integrand has degree 3N - 1 per direction, the GLL rule is exact to 2N - 1)
or on M = floor(3(N+1)/2) Gauss-Legendre points per direction (the 3/2 rule:
exact to 2M - 1 >= 3N + 1 on affine elements).  u and T are interpolated to
the quadrature points from the nodal values; grad T = sum_a grad r_a dT/dr_a
with the metric of the element map interpolated the same way.  With
G_ad = w detJ dr_a/dx_d at each point (nine factors), the integrand is
sum_d u_d sum_a G_ad dT/dr_a.
"""

from __future__ import annotations

import numpy as np

from .geometry import tensor
from .gll import gll_nodes_weights, deriv_matrix


def dealias_points(N: int) -> int:
    """Gauss-Legendre points per direction of the 3/2 rule."""
    return (3 * (N + 1)) // 2


def lagrange_at(x_nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(len(x), len(x_nodes)): the Lagrange basis of x_nodes at the points x
    (product formula)."""
    n = x_nodes.size
    L = np.ones((x.size, n))
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] *= (x - x_nodes[m]) / (x_nodes[j] - x_nodes[m])
    return L


def _apply3(Mk, Mj, Mi, X):
    """(Mk x Mj x Mi) on element blocks X (E, nk*nj*ni) in [k][j][i] order."""
    E = X.shape[0]
    T = X.reshape(E, Mk.shape[1], Mj.shape[1], Mi.shape[1])
    T = np.einsum("ai,ekji->ekja", Mi, T)
    T = np.einsum("bj,ekja->ekba", Mj, T)
    T = np.einsum("ck,ekba->ecba", Mk, T)
    return T.reshape(E, -1)


def quadrature(N: int, dealias: bool):
    """(points, weights, J, JD): the rule, the interpolation J from the GLL
    nodes to it and the interpolated derivative JD = J D (J = I, JD = D on
    the GLL nodes)."""
    xg, _ = gll_nodes_weights(N)
    D = deriv_matrix(N)
    if not dealias:
        _, w = gll_nodes_weights(N)
        return xg, w, np.eye(N + 1), D
    M = dealias_points(N)
    xq, w = np.polynomial.legendre.leggauss(M)
    J = lagrange_at(xg, xq)
    return xq, w, J, J @ D


def geometric_factors_q(xyz: np.ndarray, N: int, dealias: bool) -> np.ndarray:
    """(E, 3, 3, Q): G_ad = w detJ dr_a/dx_d at the quadrature points."""
    _, w, J, JD = quadrature(N, dealias)
    E = xyz.shape[0]
    dX = np.empty((E, 3, 3, w.size ** 3))  # dX[e, c, a] = d x_c / d r_a
    for c in range(3):
        xc = np.ascontiguousarray(xyz[:, :, c])
        dX[:, c, 0] = _apply3(J, J, JD, xc)
        dX[:, c, 1] = _apply3(J, JD, J, xc)
        dX[:, c, 2] = _apply3(JD, J, J, xc)
    Jm = np.moveaxis(dX, 3, 1)  # (E, Q, 3, 3): [c][a]
    det = np.linalg.det(Jm)
    inv = np.linalg.inv(Jm)  # [a][c] = d r_a / d x_c
    W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
    return np.moveaxis(inv * (W * det)[..., None, None], 1, 3)  # (E, 3(a), 3(d), Q)


def convect(u: np.ndarray, T: np.ndarray, xyz: np.ndarray, N: int, dealias: bool = True):
    """C_e(u) T on every element (unassembled): u (E, P, 3), T (E, P) -> (E, P)."""
    _, _, J, JD = quadrature(N, dealias)
    G = geometric_factors_q(xyz, N, dealias)
    Ta = [_apply3(J, J, JD, T), _apply3(J, JD, J, T), _apply3(JD, J, J, T)]
    uq = [_apply3(J, J, J, np.ascontiguousarray(u[:, :, d])) for d in range(3)]
    c = sum(uq[d] * sum(G[:, a, d] * Ta[a] for a in range(3)) for d in range(3))
    return _apply3(J.T, J.T, J.T, c)

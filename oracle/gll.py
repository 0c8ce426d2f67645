"""O1/O2: Gauss-Lobatto-Legendre nodes, weights and derivative matrix.

Test infrastructure only (see the package docstring).

The method collocates a nodal Lagrange basis and its quadrature on the GLL
points (Sec. 2.2).  Textbook definitions used here:

* nodes: xi_0 = -1, xi_N = +1, interior nodes = roots of P_N'(xi), found by
  Newton's method on q(xi) = (1 - xi^2) P_N'(xi) = N (P_{N-1}(xi) - xi P_N(xi)),
  whose derivative is -N(N+1) P_N(xi) (Legendre's equation), started from
  -cos(pi j / N);
* weights: rho_j = 2 / (N (N+1) P_N(xi_j)^2);
* derivative matrix D_ij = l_j'(xi_i):
  D_ij = P_N(xi_i) / (P_N(xi_j) (xi_i - xi_j)) for i != j,
  D_00 = -N(N+1)/4, D_NN = +N(N+1)/4, all other diagonal entries 0.
"""

from __future__ import annotations

import numpy as np


def legendre(N: int, x):
    """(P_N(x), P_{N-1}(x)) by the three-term recurrence
    (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if N == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    for m in range(1, N):
        p_prev, p = p, ((2 * m + 1) * x * p - m * p_prev) / (m + 1)
    return p, p_prev


def gll_nodes_weights(N: int) -> tuple[np.ndarray, np.ndarray]:
    """GLL nodes (ascending) and weights for order N >= 1."""
    if N < 1:
        raise ValueError("N >= 1 required")
    j = np.arange(N + 1)
    xi = -np.cos(np.pi * j / N)
    for _ in range(100):
        pN, pNm1 = legendre(N, xi)
        # Newton step on q = N (P_{N-1} - xi P_N), q' = -N (N+1) P_N
        step = (pNm1 - xi * pN) / ((N + 1) * pN)
        step[0] = step[-1] = 0.0
        xi = xi + step
        if np.max(np.abs(step)) < 1e-16:
            break
    xi[0], xi[-1] = -1.0, 1.0
    pN, _ = legendre(N, xi)
    rho = 2.0 / (N * (N + 1) * pN ** 2)
    return xi, rho


def deriv_matrix(N: int) -> np.ndarray:
    """D_ij = l_j'(xi_i) from the closed form in Legendre values."""
    xi, _ = gll_nodes_weights(N)
    pN, _ = legendre(N, xi)
    n = N + 1
    D = np.zeros((n, n))
    for i in range(n):
        for jj in range(n):
            if i != jj:
                D[i, jj] = pN[i] / (pN[jj] * (xi[i] - xi[jj]))
    D[0, 0] = -N * (N + 1) / 4.0
    D[N, N] = N * (N + 1) / 4.0
    return D


def deriv_matrix_barycentric(xi: np.ndarray) -> np.ndarray:
    """Independent construction of the Lagrange derivative matrix on arbitrary
    distinct nodes by barycentric weights w_j = 1 / prod_{k != j}(xi_j - xi_k):
    D_ij = (w_j / w_i) / (xi_i - xi_j), D_ii = -sum_{j != i} D_ij."""
    n = xi.size
    w = np.array([1.0 / np.prod([xi[j] - xi[k] for k in range(n) if k != j]) for j in range(n)])
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (w[j] / w[i]) / (xi[i] - xi[j])
        D[i, i] = -np.sum(D[i, :])
    return D

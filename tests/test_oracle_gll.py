"""Pins of the oracle's GLL nodes, weights and derivative matrix (O1, O2).

The method's nodal basis and quadrature are the Gauss-Lobatto-Legendre
points (Sec. 2.2).  Pins: textbook closed forms for N = 1..4, numpy's Legendre
root finder, polynomial exactness of the quadrature and of differentiation,
and an independent barycentric construction of D.
"""

import numpy as np
import pytest
from numpy.polynomial import legendre as L

import oracle

CLOSED = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / np.sqrt(5), 1 / np.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -np.sqrt(3 / 7), 0.0, np.sqrt(3 / 7), 1.0],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_closed_forms(N):
    xi, rho = oracle.gll_nodes_weights(N)
    np.testing.assert_allclose(xi, CLOSED[N][0], atol=1e-15)
    np.testing.assert_allclose(rho, CLOSED[N][1], rtol=1e-14)


@pytest.mark.parametrize("N", range(2, 13))
def test_gll_interior_nodes_are_legendre_derivative_roots(N):
    c = np.zeros(N + 1)
    c[N] = 1.0
    roots = np.sort(np.real(L.legroots(L.legder(c))))
    xi, _ = oracle.gll_nodes_weights(N)
    np.testing.assert_allclose(xi[1:-1], roots, atol=1e-13)


@pytest.mark.parametrize("N", range(1, 13))
def test_gll_symmetry_and_weight_sum(N):
    xi, rho = oracle.gll_nodes_weights(N)
    np.testing.assert_allclose(xi, -xi[::-1], atol=1e-15)
    np.testing.assert_allclose(rho, rho[::-1], rtol=1e-13)
    assert abs(rho.sum() - 2.0) < 1e-13
    assert np.all(np.diff(xi) > 0)


@pytest.mark.parametrize("N", range(1, 12))
def test_gll_quadrature_exact_to_2N_minus_1_not_2N(N):
    xi, rho = oracle.gll_nodes_weights(N)
    for m in range(0, 2 * N):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(rho @ xi ** m - exact) < 1e-13, m
    m = 2 * N
    assert rho @ xi ** m - 2.0 / (m + 1) > 1e-8  # GLL over-integrates x^(2N)


def test_deriv_matrix_closed_form_N2():
    D = oracle.deriv_matrix(2)
    ref = np.array([[-1.5, 2.0, -0.5], [-0.5, 0.0, 0.5], [0.5, -2.0, 1.5]])
    np.testing.assert_allclose(D, ref, atol=1e-15)


@pytest.mark.parametrize("N", range(1, 13))
def test_deriv_matrix_exact_on_monomials(N):
    xi, _ = oracle.gll_nodes_weights(N)
    D = oracle.deriv_matrix(N)
    for m in range(0, N + 1):
        d = m * xi ** (m - 1) if m > 0 else np.zeros_like(xi)
        np.testing.assert_allclose(D @ xi ** m, d, atol=1e-13 * N * N)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-12 * N)


@pytest.mark.parametrize("N", range(1, 13))
def test_deriv_matrix_matches_barycentric(N):
    xi, _ = oracle.gll_nodes_weights(N)
    np.testing.assert_allclose(oracle.deriv_matrix(N), oracle.deriv_matrix_barycentric(xi),
                               atol=1e-12 * N * N)


def test_deriv_matrix_corners():
    for N in range(1, 11):
        D = oracle.deriv_matrix(N)
        assert D[0, 0] == -N * (N + 1) / 4 and D[N, N] == N * (N + 1) / 4
        assert np.all(np.diag(D)[1:-1] == 0.0)

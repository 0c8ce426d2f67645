"""Pins of the oracle's geometry and element operator (O3, O4, O7, backward).

The operator is the matrix-free tensor-product form of the weak Laplacian /
Helmholtz operator carried to deformed elements by the chain rule (Sec. 2.2).
Pins: brick closed forms (geometry, Kronecker form of the element matrix,
exact energy and mass integrals of polynomials), volume, constants in the
kernel, the patch test, symmetry, the diagonal against the dense matrix, and
the dot-product identity of the k-backward contraction.
"""

import numpy as np
import pytest
from numpy.polynomial import Polynomial

import oracle
from oracle.geometry import geometric_factors
from oracle.operator import local_apply, local_diagonal, kgrad_contraction
from sem_inputs import box_mesh, random_local_normal


def brick(N, lo=(0.2, -0.1, 0.5), h=(0.7, 1.3, 0.4)):
    xi, _ = oracle.gll_nodes_weights(N)
    m = box_mesh(N, (1, 1, 1), lengths=h, dirichlet="none", ref_nodes=xi)
    xyz = m.xyz + np.array(lo)
    return xyz, m


@pytest.mark.parametrize("N", [1, 2, 3, 7])
def test_brick_geometric_factors(N):
    h = (0.7, 1.3, 0.4)
    xyz, _ = brick(N, h=h)
    G, B, detJ = geometric_factors(xyz, N)
    _, rho = oracle.gll_nodes_weights(N)
    w = np.einsum("k,j,i->kji", rho, rho, rho).ravel()
    hx, hy, hz = h
    np.testing.assert_allclose(G[0, 0], w * hy * hz / (2 * hx), rtol=1e-13)
    np.testing.assert_allclose(G[0, 3], w * hx * hz / (2 * hy), rtol=1e-13)
    np.testing.assert_allclose(G[0, 5], w * hx * hy / (2 * hz), rtol=1e-13)
    for c in (1, 2, 4):
        assert np.max(np.abs(G[0, c])) < 1e-14
    np.testing.assert_allclose(B[0], w * hx * hy * hz / 8, rtol=1e-13)


@pytest.mark.parametrize("N,shape,lengths,z_ratio,volume", [
    (2, (3, 3, 3), (1.0, 1.0, 1.0), None, 1.0),
    (7, (4, 4, 4), (1.0, 1.0, 1.0), None, 1.0),
    (4, (4, 4, 4), (4.0, 4.0, 1.0), 20.0, 16.0),
])
def test_mass_sums_to_volume_on_jittered_trilinear(N, shape, lengths, z_ratio, volume):
    xi, _ = oracle.gll_nodes_weights(N)
    m = box_mesh(N, shape, lengths, jitter=0.05, z_ratio=z_ratio, ref_nodes=xi)
    G, B, detJ = geometric_factors(m.xyz, N)
    assert np.all(detJ > 0)
    assert abs(B.sum() - volume) < 1e-12 * volume


@pytest.mark.parametrize("deform", [None, dict(a=0.15, seed=1, kind="periodic")])
def test_constants_in_kernel(deform):
    N = 5
    m = box_mesh(N, (3, 3, 4), (4.0, 4.0, 1.0), periodic=(True, True, False), dirichlet="z",
                 jitter=0.0 if deform else 0.05, z_ratio=20.0, deform=deform)
    G, B, _ = geometric_factors(m.xyz, N)
    w = local_apply(np.ones((m.E, m.P)), G, B, N)
    assert np.max(np.abs(w)) < 1e-12 * np.max(np.abs(G))


@pytest.mark.parametrize("N", [2, 3, 6])
def test_patch_test_linear_fields(N):
    """Q^T A_L Q x_lin vanishes at interior unique nodes of trilinear meshes
    (quadrature exact: integrand degree <= N+1 <= 2N-1 per variable)."""
    xi, _ = oracle.gll_nodes_weights(N)
    m = box_mesh(N, (3, 3, 3), jitter=0.05, ref_nodes=xi)
    G, B, _ = geometric_factors(m.xyz, N)
    num = oracle.Numbering(m.gid, m.dirichlet)
    for d in range(3):
        w = num.Qt(local_apply(np.ascontiguousarray(m.xyz[..., d]), G, B, N))
        interior = ~num.dirichlet_u
        assert np.max(np.abs(w[interior])) < 1e-12, d


def test_patch_test_detects_a_planted_cross_term_error():
    """Dropping the G_rt cross term from both v_r and v_t keeps symmetry but
    must fail the patch test on a jittered mesh."""
    N = 3
    xi, _ = oracle.gll_nodes_weights(N)
    m = box_mesh(N, (3, 3, 3), jitter=0.05, ref_nodes=xi)
    G, B, _ = geometric_factors(m.xyz, N)
    G2 = G.copy()
    G2[:, 2, :] = 0.0
    num = oracle.Numbering(m.gid, m.dirichlet)
    w = num.Qt(local_apply(np.ascontiguousarray(m.xyz[..., 0]), G2, B, N))
    assert np.max(np.abs(w[~num.dirichlet_u])) > 1e-6


@pytest.mark.parametrize("N", [1, 2, 4, 7])
def test_brick_kronecker_form(N):
    h = (0.7, 1.3, 0.4)
    xyz, _ = brick(N, h=h)
    G, B, _ = geometric_factors(xyz, N)
    A = oracle.element_matrices(G, B, N)[0]
    _, rho = oracle.gll_nodes_weights(N)
    D = oracle.deriv_matrix(N)
    K = D.T @ np.diag(rho) @ D
    M = np.diag(rho)
    hx, hy, hz = h
    ref = (hy * hz / (2 * hx) * np.kron(M, np.kron(M, K))
           + hx * hz / (2 * hy) * np.kron(M, np.kron(K, M))
           + hx * hy / (2 * hz) * np.kron(K, np.kron(M, M)))
    np.testing.assert_allclose(A, ref, atol=1e-13 * np.abs(ref).max())


def _poly_on(deg, seed):
    return Polynomial(np.random.default_rng(seed).standard_normal(deg + 1))


@pytest.mark.parametrize("N", [2, 4, 7])
def test_brick_energy_and_mass_of_polynomials_exact(N):
    lo, h = (0.2, -0.1, 0.5), (0.7, 1.3, 0.4)
    xyz, _ = brick(N, lo=lo, h=h)
    G, B, _ = geometric_factors(xyz, N)
    p, q, s = _poly_on(N - 1, 1), _poly_on(N - 1, 2), _poly_on(N - 1, 3)
    x, y, z = xyz[0, :, 0], xyz[0, :, 1], xyz[0, :, 2]
    u = (p(x) * q(y) * s(z))[None, :]

    def integ(poly, a, b):
        P = poly.integ()
        return P(b) - P(a)

    ax_, bx = lo[0], lo[0] + h[0]
    ay, by = lo[1], lo[1] + h[1]
    az, bz = lo[2], lo[2] + h[2]
    Ip2, Iq2, Is2 = integ(p * p, ax_, bx), integ(q * q, ay, by), integ(s * s, az, bz)
    Idp2 = integ(p.deriv() ** 2, ax_, bx)
    Idq2 = integ(q.deriv() ** 2, ay, by)
    Ids2 = integ(s.deriv() ** 2, az, bz)
    energy = Idp2 * Iq2 * Is2 + Ip2 * Idq2 * Is2 + Ip2 * Iq2 * Ids2
    uAu = float(u.ravel() @ local_apply(u, G, B, N).ravel())
    assert abs(uAu - energy) < 1e-12 * abs(energy)
    mass = Ip2 * Iq2 * Is2
    assert abs(float(u.ravel() @ (B * u).ravel()) - mass) < 1e-12 * abs(mass)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_element_matrix_symmetric_with_k_and_h2(N):
    m = box_mesh(N, (2, 2, 2), jitter=0.05, deform=dict(a=0.15, seed=4, kind="walls"))
    G, B, _ = geometric_factors(m.xyz, N)
    k = np.exp(0.3 * random_local_normal((m.E, m.P), 9))
    A = oracle.element_matrices(G, B, N, k=k, h2=0.7)
    for e in range(m.E):
        np.testing.assert_allclose(A[e], A[e].T, atol=1e-14 * np.abs(A[e]).max())
    # diagonal formula
    d = local_diagonal(G, B, N, k=k, h2=0.7)
    np.testing.assert_allclose(d, np.einsum("eqq->eq", A), rtol=1e-13)


def test_kbar_dot_product_identity():
    N = 4
    m = box_mesh(N, (2, 2, 2), jitter=0.05)
    G, B, _ = geometric_factors(m.xyz, N)
    u = random_local_normal((m.E, m.P), 1)
    wb = random_local_normal((m.E, m.P), 2)
    dk = random_local_normal((m.E, m.P), 3)
    lhs = np.sum(wb * local_apply(u, G, B, N, k=dk))
    rhs = np.sum(dk * kgrad_contraction(u, wb, G, N))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # symmetry of A_L with a positive k
    k = np.exp(dk)
    a = np.sum(wb * local_apply(u, G, B, N, k=k, h2=0.3))
    b = np.sum(u * local_apply(wb, G, B, N, k=k, h2=0.3))
    assert abs(a - b) < 1e-12 * abs(a)

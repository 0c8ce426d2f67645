"""Pins of the oracle's convective operator (the advection term of the
Boussinesq equations, Sec. 2.3; readings in oracle/advection.py).

Pins: on affine (brick) elements the 3/2-rule result equals a brute-force
Gauss quadrature of phi_i u . grad T with the analytic gradient of global
polynomial fields (the 3/2 rule is exact there, the GLL collocation is not);
the collocation variant equals B u . grad T at the nodes; on a periodic box
the assembled operator with a constant velocity is skew: T . C(u) T = 0.
"""

import numpy as np
import pytest

from oracle.advection import convect, dealias_points, lagrange_at
from oracle.assembly import Numbering
from oracle.geometry import geometric_factors
from oracle.gll import gll_nodes_weights
from sem_inputs import box_mesh


def _poly_fields(N, seed):
    """Global polynomials of degree N per variable: T and u (3 components),
    with analytic gradient of T."""
    rng = np.random.default_rng(seed)
    cT = rng.standard_normal((3, N + 1))
    cu = rng.standard_normal((3, 3, N + 1))
    P = np.polynomial.polynomial
    T = lambda X: np.prod([P.polyval(X[..., d], cT[d]) for d in range(3)], axis=0)

    def gradT(X):
        v = [P.polyval(X[..., d], cT[d]) for d in range(3)]
        dv = [P.polyval(X[..., d], P.polyder(cT[d])) for d in range(3)]
        return np.stack([dv[0] * v[1] * v[2], v[0] * dv[1] * v[2], v[0] * v[1] * dv[2]], -1)

    def U(X):
        return np.stack([np.prod([P.polyval(X[..., d], cu[c, d]) for d in range(3)], axis=0)
                         for c in range(3)], -1)
    return T, gradT, U


@pytest.mark.parametrize("N", [2, 4, 7])
def test_dealiased_convection_is_exact_on_bricks(N):
    lo = np.array([0.1, -0.2, 0.3])
    h = np.array([0.6, 0.9, 0.4])
    xi, _ = gll_nodes_weights(N)
    m = box_mesh(N, (2, 1, 2), tuple(2 * h), dirichlet="none", ref_nodes=xi)
    xyz = m.xyz + lo
    T, gradT, U = _poly_fields(N, 1)
    got = convect(U(xyz), T(xyz), xyz, N, dealias=True)
    # brute force: tensor Gauss rule with 2N + 2 points per direction on each brick
    Q = 2 * N + 2
    xq, wq = np.polynomial.legendre.leggauss(Q)
    L = lagrange_at(xi, xq)  # basis at the rule's points
    ref = np.zeros_like(got)
    for e in range(m.E):
        X0 = xyz[e].reshape(N + 1, N + 1, N + 1, 3)
        a, b = X0[0, 0, 0], X0[N, N, N]
        half = (b - a) / 2
        pts = np.stack(np.meshgrid(a[2] + half[2] * (xq + 1), a[1] + half[1] * (xq + 1),
                                   a[0] + half[0] * (xq + 1), indexing="ij"), -1)[..., ::-1]
        f = np.sum(U(pts) * gradT(pts), -1) * np.prod(half)
        W = np.einsum("k,j,i->kji", wq, wq, wq)
        ref[e] = np.einsum("ck,bj,ai,kji->cba", L.T, L.T, L.T, W * f).reshape(-1)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-11 * scale
    alias = convect(U(xyz), T(xyz), xyz, N, dealias=False)
    assert np.abs(alias - ref).max() >= 1e-4 * scale  # GLL collocation is not exact


@pytest.mark.parametrize("N", [3, 6])
def test_collocation_equals_mass_times_pointwise_convection(N):
    m = box_mesh(N, (2, 2, 1), (1.2, 0.8, 0.5), dirichlet="none")
    T, gradT, U = _poly_fields(N, 2)
    got = convect(U(m.xyz), T(m.xyz), m.xyz, N, dealias=False)
    _, B, _ = geometric_factors(m.xyz, N)
    want = B * np.sum(U(m.xyz) * gradT(m.xyz), -1)
    np.testing.assert_allclose(got, want, atol=1e-11 * np.abs(want).max())


@pytest.mark.parametrize("dealias", [True, False])
def test_constant_velocity_convection_is_skew_on_a_periodic_box(dealias):
    N = 5
    m = box_mesh(N, (3, 3, 2), (1.0, 1.0, 1.0), periodic=(True, True, True), dirichlet="none")
    num = Numbering(m.gid)
    Tu = np.random.default_rng(3).standard_normal(num.n)
    TL = num.Q(Tu)
    u = np.broadcast_to(np.array([0.7, -0.4, 1.3]), m.xyz.shape).copy()
    CT = num.Qt(convect(u, TL, m.xyz, N, dealias=dealias))
    assert abs(Tu @ CT) <= 1e-12 * np.linalg.norm(Tu) * np.linalg.norm(CT)


def test_dealias_points():
    assert [dealias_points(N) for N in (1, 5, 7, 9, 10)] == [3, 9, 12, 15, 16]

"""Pins of the oracle's convective operator (the advection term of the
Boussinesq equations, Sec. 4.1; readings in oracle/advection.py).

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


# ---------------------------------------------------------------- general maps
# On the bricks above dr_a/dx_d is diagonal, so an index mistake in the metric
# (a and d swapped, the adjugate transposed) would not show.  The pins below
# use affine elements x = c + M r with a full, non-symmetric M (rotated and
# sheared), and jittered, deformed meshes.

def _affine_elements(N, n_el, seed):
    """n_el separate affine elements x = c_e + M_e r (det M_e > 0) at the GLL
    nodes: xyz (E, P, 3), the maps M (E, 3, 3), the reference points (P, 3)."""
    rng = np.random.default_rng(seed)
    xi, _ = gll_nodes_weights(N)
    k, j, i = np.meshgrid(xi, xi, xi, indexing="ij")
    r = np.stack([i.ravel(), j.ravel(), k.ravel()], -1)  # q = i + n (j + n k)
    Ms = []
    for _ in range(n_el):
        Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
        Q = Q * np.sign(np.diag(R))
        if np.linalg.det(Q) < 0:
            Q[:, 0] = -Q[:, 0]
        S = np.diag(rng.uniform(0.3, 0.7, 3))
        S[0, 1], S[0, 2], S[1, 2] = rng.uniform(-0.25, 0.25, 3)
        Ms.append(Q @ S)
    M = np.array(Ms)
    c = rng.uniform(-1.0, 1.0, (n_el, 3))
    xyz = c[:, None, :] + np.einsum("ecd,qd->eqc", M, r)
    return xyz, M, r


def _ref_poly(N, seed):
    """A field that is a polynomial of degree <= N in each reference
    coordinate (a sum of two tensor products), with its reference gradient."""
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((2, 3, N + 1))
    P = np.polynomial.polynomial

    def f(r):
        return sum(np.prod([P.polyval(r[..., d], C[t, d]) for d in range(3)], axis=0)
                   for t in range(2))

    def grad(r):
        g = np.zeros(r.shape)
        for t in range(2):
            v = [P.polyval(r[..., d], C[t, d]) for d in range(3)]
            dv = [P.polyval(r[..., d], P.polyder(C[t, d])) for d in range(3)]
            g[..., 0] += dv[0] * v[1] * v[2]
            g[..., 1] += v[0] * dv[1] * v[2]
            g[..., 2] += v[0] * v[1] * dv[2]
        return g
    return f, grad


def _affine_convection_error(N, conv):
    """max |conv - brute force| / max |brute force| on sheared affine
    elements, where the brute force is a tensor Gauss rule of 2N + 2 points
    per direction in reference coordinates with the chain-rule gradient
    grad_x T = M^-T grad_r T and detJ = det M (exact for these integrands)."""
    xyz, M, r = _affine_elements(N, 3, seed=10 + N)
    E = xyz.shape[0]
    T, gT = _ref_poly(N, 20 + N)
    U = [_ref_poly(N, 30 + N + c)[0] for c in range(3)]
    T_n = np.tile(T(r), (E, 1))
    u_n = np.tile(np.stack([U[c](r) for c in range(3)], -1), (E, 1, 1))
    got = conv(u_n, T_n, xyz, N)
    Q = 2 * N + 2
    xq, wq = np.polynomial.legendre.leggauss(Q)
    k, j, i = np.meshgrid(xq, xq, xq, indexing="ij")
    rq = np.stack([i.ravel(), j.ravel(), k.ravel()], -1)
    W = np.einsum("k,j,i->kji", wq, wq, wq).ravel()
    xi, _ = gll_nodes_weights(N)
    L = lagrange_at(xi, xq)  # (Q, N+1)
    phi = np.einsum("ck,bj,ai->cbakji", L.T, L.T, L.T).reshape((N + 1) ** 3, Q ** 3)
    uq = np.stack([U[c](rq) for c in range(3)], -1)
    ref = np.empty_like(got)
    for e in range(E):
        gx = np.linalg.solve(M[e].T, gT(rq).T).T  # grad_x T = M^-T grad_r T
        ref[e] = phi @ (W * np.sum(uq * gx, -1) * np.linalg.det(M[e]))
    return np.abs(got - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("N", [2, 4, 7])
def test_dealiased_convection_is_exact_on_sheared_affine_elements(N):
    err = _affine_convection_error(N, lambda u, T, x, n: convect(u, T, x, n, dealias=True))
    assert err <= 1e-11, err


def test_affine_pin_detects_a_planted_transposed_metric(monkeypatch):
    """The metric with a and d swapped (dr_d/dx_a in place of dr_a/dx_d)
    agrees on bricks but must fail the sheared-element pin."""
    import oracle.advection as adv

    good = adv.geometric_factors_q
    monkeypatch.setattr(adv, "geometric_factors_q",
                        lambda xyz, N, dealias: np.swapaxes(good(xyz, N, dealias), 1, 2))
    err = _affine_convection_error(4, lambda u, T, x, n: adv.convect(u, T, x, n, dealias=True))
    assert err > 1e-3, err
    # the coordinate-field identity below catches it on a deformed mesh too
    N = 3
    md = box_mesh(N, (2, 2, 2), (1.0, 1.2, 0.8), dirichlet="none", jitter=0.08, jitter_seed=4,
                  deform=dict(a=0.2, seed=5, kind="walls"))
    u = np.zeros(md.xyz.shape)
    u[..., 1] = 1.0
    off = adv.convect(u, np.ascontiguousarray(md.xyz[..., 0]), md.xyz, N, dealias=True)
    assert np.abs(off).max() > 1e-4


@pytest.mark.parametrize("dealias", [True, False])
@pytest.mark.parametrize("N", [3, 7])
def test_coordinate_fields_give_the_weighted_jacobian_identity(N, dealias):
    """T = x_c and u = e_d (constant): the integrand is w detJ
    sum_a (dr_a/dx_d)(dx_c/dr_a) = w detJ delta_cd, so C(e_d) x_c = 0 for
    c != d (any element map); for c = d the entries sum to sum_q w_q detJ_q,
    which on trilinear (jittered) elements with N >= 2 is their volume
    exactly (detJ has degree <= 2 per direction there)."""
    m = box_mesh(N, (2, 2, 2), (1.0, 1.2, 0.8), dirichlet="none", jitter=0.08, jitter_seed=4)
    vol = 1.0 * 1.2 * 0.8
    md = box_mesh(N, (2, 2, 2), (1.0, 1.2, 0.8), dirichlet="none", jitter=0.08, jitter_seed=4,
                  deform=dict(a=0.2, seed=5, kind="walls"))
    for mesh, exact_vol in ((m, True), (md, False)):
        scale = 0.0
        for d in range(3):
            u = np.zeros(mesh.xyz.shape)
            u[..., d] = 1.0
            for c in range(3):
                out = convect(u, np.ascontiguousarray(mesh.xyz[..., c]), mesh.xyz, N,
                              dealias=dealias)
                if c == d:
                    scale = max(scale, np.abs(out).max())
                    if exact_vol and dealias:
                        assert abs(out.sum() - vol) <= 1e-12 * vol
                    if exact_vol and not dealias:  # GLL: also exact to degree 2N - 1 >= 2
                        assert abs(out.sum() - vol) <= 1e-12 * vol
                else:
                    assert np.abs(out).max() <= 1e-12 * max(scale, 1e-3), (c, d)


@pytest.mark.parametrize("N", [3, 6])
def test_collocation_identity_on_a_deformed_mesh(N):
    """GLL collocation: C(u) T = B (u . grad T) at the nodes on a jittered,
    deformed mesh, with grad T = J^-T (D_r T, D_s T, D_t T) formed from the
    oracle's nodal Jacobian (the 3 x 3 matrix dx_c/dr_a at each node)."""
    from oracle.geometry import jacobian, tensor, d_r, d_s, d_t
    from oracle.gll import deriv_matrix

    m = box_mesh(N, (2, 2, 2), (1.0, 1.0, 1.0), dirichlet="none", jitter=0.08,
                 deform=dict(a=0.2, seed=6, kind="walls"))
    rng = np.random.default_rng(N)
    T = rng.standard_normal((m.E, m.P))
    u = rng.standard_normal((m.E, m.P, 3))
    J = jacobian(m.xyz, N)  # J[e, q, c, a] = dx_c / dr_a
    D = deriv_matrix(N)
    Tt = tensor(T, N)
    gr = np.stack([d_r(D, Tt).reshape(m.E, -1), d_s(D, Tt).reshape(m.E, -1),
                   d_t(D, Tt).reshape(m.E, -1)], -1)  # dT/dr_a
    gx = np.linalg.solve(np.swapaxes(J, -1, -2), gr[..., None])[..., 0]  # J^T gx = gr
    _, B, _ = geometric_factors(m.xyz, N)
    want = B * np.sum(u * gx, -1)
    got = convect(u, T, m.xyz, N, dealias=False)
    np.testing.assert_allclose(got, want, atol=1e-12 * np.abs(want).max())

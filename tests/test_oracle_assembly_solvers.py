"""Pins of the oracle's assembly, PCG, Chebyshev and Lanczos (O5-O11).

Pins: unique-point counts (the paper counts N_e p^3 points on the periodic
box, Sec. 4.1 / Table of simulations), multiplicities, the Kronecker-sum form
of the assembled matrix on uniform meshes built from independently assembled
1-D matrices, symmetry / definiteness / null space of explicit matrices,
agreement of CG with scipy's sparse direct solver, the fourth-kind Chebyshev
error polynomial in closed form, Lanczos against a dense eigensolver, and the
spectral convergence of the manufactured solution.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle.geometry import geometric_factors
from sem_inputs import box_mesh, config_mesh, manufactured_sine, random_local_normal


# --------------------------------------------------------------------- counts

@pytest.mark.parametrize("cfg,N,n", [(1, 7, 29 ** 3), (3, 9, 37 ** 3)])
def test_unique_counts_cube(cfg, N, n):
    m, _ = config_mesh(cfg)
    num = oracle.Numbering(m.gid, m.dirichlet)
    assert num.n == n == (4 * N + 1) ** 3
    assert num.n_free == (4 * N - 1) ** 3
    np.testing.assert_array_equal(num.Qt(np.ones(m.gid.shape)), num.mult)
    assert num.mult.sum() == m.E * m.P


def test_unique_counts_periodic_box_match_paper_convention():
    # the paper's point count N_e p^3 holds on the horizontally periodic box
    N, shape = 5, (4, 3, 2)
    m = box_mesh(N, shape, (4.0, 4.0, 1.0), periodic=(True, True, False), dirichlet="z")
    num = oracle.Numbering(m.gid, m.dirichlet)
    assert num.n == (4 * N) * (3 * N) * (2 * N + 1)
    assert num.n_free == (4 * N) * (3 * N) * (2 * N - 1)
    # the full-size box of the benchmark: 32x32x16 elements, N = 7
    assert 32 * 7 * 32 * 7 * (16 * 7 + 1) == 5669888


# ------------------------------------------------------------- kronecker sum

def _assemble_1d(K1, ne, h, periodic=False):
    N = K1.shape[0] - 1
    n = ne * N + (0 if periodic else 1)
    A = np.zeros((n, n))
    for e in range(ne):
        idx = [(e * N + i) % n for i in range(N + 1)]
        A[np.ix_(idx, idx)] += K1 * h
    return A


@pytest.mark.parametrize("N", [2, 4])
def test_uniform_mesh_assembled_kronecker_sum(N):
    shape, L = (3, 2, 2), (1.5, 1.0, 0.8)
    xi, rho = oracle.gll_nodes_weights(N)
    m = box_mesh(N, shape, L, periodic=(True, False, False), dirichlet="none", ref_nodes=xi)
    G, B, _ = geometric_factors(m.xyz, N)
    num = oracle.Numbering(m.gid, None)
    A = oracle.explicit_matrix(G, B, N, num, free_only=False).toarray()
    D = oracle.deriv_matrix(N)
    Khat, Mhat = D.T @ np.diag(rho) @ D, np.diag(rho)
    hx, hy, hz = (L[d] / shape[d] for d in range(3))
    Kx = _assemble_1d(Khat, shape[0], 2 / hx, periodic=True)
    Mx = _assemble_1d(Mhat, shape[0], hx / 2, periodic=True)
    Ky, My = _assemble_1d(Khat, shape[1], 2 / hy), _assemble_1d(Mhat, shape[1], hy / 2)
    Kz, Mz = _assemble_1d(Khat, shape[2], 2 / hz), _assemble_1d(Mhat, shape[2], hz / 2)
    ref = np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Kz, np.kron(My, Mx))
    # global id = gx + GX (gy + GY gz) with sorted unique ids -> same order
    np.testing.assert_allclose(A, ref, atol=1e-13 * np.abs(ref).max())


# ------------------------------------------------------------ explicit matrix

def _small_problem(N, shape=(2, 2, 2), dirichlet="all", jitter=0.05, k=False, h2=0.0, seed=1):
    m = box_mesh(N, shape, dirichlet=dirichlet, jitter=jitter, jitter_seed=seed)
    kk = np.exp(0.4 * random_local_normal((m.E, m.P), 11)) if k else None
    return m, oracle.Problem(m.xyz, m.gid, m.dirichlet, N, k=kk, h2=h2)


@pytest.mark.parametrize("N,k,h2", [(3, False, 0.0), (4, True, 1.0), (7, False, 0.0)])
def test_explicit_matrix_symmetric_spd_and_matches_apply(N, k, h2):
    m, P = _small_problem(N, k=k, h2=h2)
    A = oracle.explicit_matrix(P.G, P.B, N, P.num, k=P.k, h2=h2)
    assert spla.norm(A - A.T) <= 1e-14 * spla.norm(A)
    x = np.random.default_rng(0).standard_normal(P.num.n_free)
    np.testing.assert_allclose(A @ x, P.apply(x), atol=1e-12 * np.abs(A @ x).max())
    if P.num.n_free <= 1000:
        lam = np.linalg.eigvalsh(A.toarray())
        assert lam[0] > 0
    np.testing.assert_allclose(P.diag(), A.diagonal(), rtol=1e-13)


def test_explicit_matrix_neumann_single_null_mode():
    N = 3
    m, P = _small_problem(N, dirichlet="none")
    A = oracle.explicit_matrix(P.G, P.B, N, P.num).toarray()
    lam, V = np.linalg.eigh(A)
    scale = lam[-1]
    assert abs(lam[0]) < 1e-12 * scale and lam[1] > 1e-6 * scale
    v = V[:, 0] / V[0, 0]
    np.testing.assert_allclose(v, 1.0, atol=1e-10)


# ------------------------------------------------------------------------ CG

@pytest.mark.parametrize("N,shape", [(4, (2, 2, 2)), (3, (3, 3, 3)), (7, (2, 2, 2))])
def test_pcg_matches_sparse_direct_solve(N, shape):
    m, P = _small_problem(N, shape=shape, k=True, h2=0.5)
    A = oracle.explicit_matrix(P.G, P.B, N, P.num, k=P.k, h2=0.5).tocsc()
    b = np.random.default_rng(3).standard_normal(P.num.n_free)
    x_ref = spla.spsolve(A, b)
    res = P.solve(b, rtol=1e-13)
    assert res["converged"]
    assert np.linalg.norm(res["x"] - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    res2 = P.solve(b, rtol=1e-13, precond="chebyshev")
    assert res2["converged"] and res2["iters"] < res["iters"]
    assert np.linalg.norm(res2["x"] - x_ref) <= 1e-10 * np.linalg.norm(x_ref)


def test_neumann_solve_matches_least_squares():
    N = 3
    m, P = _small_problem(N, dirichlet="none")
    A = oracle.explicit_matrix(P.G, P.B, N, P.num).toarray()
    b = np.random.default_rng(4).standard_normal(P.num.n)
    b -= b.mean()
    x_ref = np.linalg.lstsq(A, b, rcond=None)[0]
    x_ref -= x_ref.mean()
    res = P.solve(b, rtol=1e-12)
    assert res["converged"]
    assert abs(res["x"].mean()) < 1e-14 * np.abs(res["x"]).max()
    assert np.linalg.norm(res["x"] - x_ref) <= 1e-9 * np.linalg.norm(x_ref)


def test_fixed_iteration_mode_runs_exactly():
    m, P = _small_problem(4)
    b = np.random.default_rng(5).standard_normal(P.num.n_free)
    res = P.solve(b, rtol=1e-30, max_iter=17, fixed_iters=True)
    assert res["iters"] == 17 and res["res_hist"].size == 18


# ----------------------------------------------------------------- Chebyshev

def _w4(m, x):
    """Fourth-kind Chebyshev polynomial W_m(cos t) = sin((m + 1/2) t) / sin(t / 2)."""
    t = np.arccos(np.clip(x, -1.0, 1.0))
    out = np.empty_like(t)
    small = np.abs(np.sin(t / 2)) < 1e-14
    out[~small] = np.sin((m + 0.5) * t[~small]) / np.sin(t[~small] / 2)
    out[small] = 2 * m + 1
    return out


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_chebyshev_error_polynomial_closed_form(m):
    lam = np.linspace(1e-4, 1.0, 257)
    rho_hat = 1.0
    z = oracle.chebyshev_apply(lambda v: lam * v, np.ones_like(lam), np.ones_like(lam), m, rho_hat)
    e = 1.0 - lam * z
    np.testing.assert_allclose(e, _w4(m, 1.0 - 2.0 * lam / rho_hat) / (2 * m + 1), atol=1e-13)
    assert np.all(np.abs(e) < 1.0)
    assert abs(abs(e[-1]) - 1.0 / (2 * m + 1)) < 1e-13


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8])
def test_first_kind_chebyshev_error_polynomial_closed_form(m):
    """Classical semi-iteration on [rho/10, rho]: 1 - lam p(lam) equals
    T_m((theta - lam)/delta) / T_m(theta/delta) (numpy's Chebyshev series)."""
    from numpy.polynomial import chebyshev as C
    rho_hat = 1.7
    lo, hi = rho_hat / 10, rho_hat
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    lam = np.linspace(1e-4, rho_hat, 301)
    z = oracle.chebyshev1_apply(lambda v: lam * v, np.ones_like(lam), np.ones_like(lam), m, rho_hat)
    Tm = np.zeros(m + 1)
    Tm[m] = 1.0
    expect = C.chebval((theta - lam) / delta, Tm) / C.chebval(theta / delta, Tm)
    np.testing.assert_allclose(1.0 - lam * z, expect, atol=1e-12)
    inside = lam >= lo
    assert np.all(np.abs(1.0 - lam[inside] * z[inside]) <= 1.0 / C.chebval(theta / delta, Tm) + 1e-12)


def test_first_kind_chebyshev_pcg_converges_to_the_jacobi_solution():
    N = 3
    m, P = _small_problem(N, k=True, h2=0.2)
    b = np.random.default_rng(8).standard_normal(P.num.n_free)
    ref = P.solve(b, rtol=1e-12)
    res = P.solve(b, rtol=1e-10, precond="chebyshev1", m=4)
    assert res["converged"] and res["iters"] < ref["iters"]
    assert np.linalg.norm(res["x"] - ref["x"]) <= 1e-8 * np.linalg.norm(ref["x"])


def test_chebyshev_symmetric_and_contracting_on_operator():
    N = 3
    m, P = _small_problem(N, k=True, h2=0.2)
    A = oracle.explicit_matrix(P.G, P.B, N, P.num, k=P.k, h2=0.2).toarray()
    d = np.diag(A)
    S12 = np.diag(d ** -0.5)
    lam = np.linalg.eigvalsh(S12 @ A @ S12)
    rho_hat = 1.1 * lam[-1]
    rng = np.random.default_rng(6)
    x, y = rng.standard_normal(d.size), rng.standard_normal(d.size)
    M = lambda r: oracle.chebyshev_apply(P.apply, 1.0 / d, r, 3, rho_hat)
    assert abs(M(x) @ y - x @ M(y)) < 1e-12 * abs(M(x) @ y)
    e = _w4(3, 1.0 - 2.0 * lam / rho_hat) / 7.0
    assert np.all(np.abs(e) < 1.0)


def test_lanczos_lmax_against_dense_eigensolver():
    N = 4
    m, P = _small_problem(N, shape=(3, 3, 3), k=True, h2=0.0)
    A = oracle.explicit_matrix(P.G, P.B, N, P.num, k=P.k).toarray()
    d = np.diag(A)
    lmax = sla.eigh(A, np.diag(d), eigvals_only=True)[-1]
    est = oracle.lanczos_lmax(P.apply, 1.0 / d, np.random.default_rng(7).standard_normal(d.size), 20)
    assert est <= lmax * (1 + 1e-12)
    assert est >= 0.97 * lmax


# --------------------------------------------------------- manufactured case

@pytest.mark.slow
def test_spectral_convergence_in_N_on_config1_recipe():
    errs = []
    for N in range(2, 11):
        m, fld = config_mesh(1, N=N)
        P = oracle.Problem(m.xyz, m.gid, m.dirichlet, N)
        f = fld["f"] * 3 * np.pi ** 2
        res = P.solve(P.rhs_from_source(f), rtol=1e-13, max_iter=20000)
        uex = P.num.from_local_consistent(fld["f"])
        errs.append(np.abs(res["x"] - uex).max())
    le = np.log10(errs)
    assert np.all(np.diff(le) < 0), errs
    slope = np.polyfit(np.arange(2, 11), le, 1)[0]
    assert slope < -0.8, slope  # exponential decay in N
    assert errs[-1] < 1e-9


def _lagrange_matrix(xi, eta):
    """I[m, j] = l_j(eta_m) for the Lagrange basis on nodes xi."""
    I = np.ones((eta.size, xi.size))
    for j in range(xi.size):
        for k in range(xi.size):
            if k != j:
                I[:, j] *= (eta - xi[k]) / (xi[j] - xi[k])
    return I


def test_algebraic_convergence_under_h_refinement_N3():
    """Error sampled between the nodes (midpoints of node intervals, where no
    nodal superconvergence applies) decays like h^(N+1) on affine meshes."""
    N, errs = 3, []
    xi, _ = oracle.gll_nodes_weights(N)
    eta = 0.5 * (xi[:-1] + xi[1:])
    I = _lagrange_matrix(xi, eta)
    for ne in (2, 4, 8):
        m = box_mesh(N, (ne, ne, ne), ref_nodes=xi)
        P = oracle.Problem(m.xyz, m.gid, m.dirichlet, N)
        f = manufactured_sine(m.xyz)
        res = P.solve(P.rhs_from_source(3 * np.pi ** 2 * f), rtol=1e-13, max_iter=20000)
        U = P.num.to_local(res["x"]).reshape(m.E, N + 1, N + 1, N + 1)
        Uh = np.einsum("ak,bj,ci,ekji->eabc", I, I, I, U)
        X = np.einsum("ak,bj,ci,ekjid->eabcd", I, I, I, m.xyz.reshape(m.E, N + 1, N + 1, N + 1, 3))
        uex = np.sin(np.pi * X[..., 0]) * np.sin(np.pi * X[..., 1]) * np.sin(np.pi * X[..., 2])
        errs.append(np.abs(Uh - uex).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - (N + 1)) < 0.5), rates

"""Pins of the oracle's p-multigrid preconditioner (Sec. 2.2's default for the
pressure solve; the readings are listed in oracle/pmg.py).

Pins: the level schedule; the 1-D interpolation reproduces polynomials of its
degree and is the identity between equal orders; the coarse mesh built from
the fine one (coordinates, global ids, Dirichlet flags) equals the mesh the
input generator builds directly at the coarse order wherever the two must
agree (trilinear elements: same coordinates; any mesh: same partition of the
local points into unknowns, same Dirichlet nodes); prolongation reproduces
coarse polynomials on an affine mesh; restriction is its transpose; the
V-cycle with an exact coarse solve is symmetric positive definite; and the
preconditioned flexible CG converges in a small fraction of the Jacobi-PCG
iterations to the same solution.
"""

import numpy as np
import pytest

import oracle
from oracle.gll import gll_nodes_weights
from oracle.pmg import (PMG, coarse_mesh, interpolation_matrix, level_orders, tensor_apply)
from sem_inputs import box_mesh, config_mesh


def test_level_orders():
    assert level_orders(7) == [7, 3, 1]
    assert level_orders(9) == [9, 4, 2, 1]
    assert level_orders(10) == [10, 5, 2, 1]
    assert level_orders(1) == [1]


@pytest.mark.parametrize("n_from,n_to", [(1, 7), (3, 7), (4, 9), (7, 3), (9, 4), (2, 2), (6, 6)])
def test_interpolation_reproduces_polynomials(n_from, n_to):
    J = interpolation_matrix(n_from, n_to)
    xf, _ = gll_nodes_weights(n_from)
    xt, _ = gll_nodes_weights(n_to)
    for m in range(n_from + 1):
        np.testing.assert_allclose(J @ xf ** m, xt ** m, atol=1e-13)
    if n_from == n_to:
        np.testing.assert_array_equal(J, np.eye(n_from + 1))
    np.testing.assert_allclose(J.sum(axis=1), 1.0, atol=1e-14)


def test_tensor_apply_reproduces_tensor_polynomials():
    n_from, n_to = 3, 6
    xf, _ = gll_nodes_weights(n_from)
    xt, _ = gll_nodes_weights(n_to)
    f = lambda r, s, t: (1 + r - 2 * r ** 3) * (s ** 2 - 0.5 * s) * (t ** 3 + t)
    T = np.meshgrid(xf, xf, xf, indexing="ij")  # [k][j][i] order: t, s, r
    Ff = f(T[2], T[1], T[0]).reshape(1, -1)
    Tt = np.meshgrid(xt, xt, xt, indexing="ij")
    Ft = f(Tt[2], Tt[1], Tt[0]).reshape(1, -1)
    np.testing.assert_allclose(tensor_apply(interpolation_matrix(n_from, n_to), Ff), Ft,
                               atol=1e-13)


def _same_partition(a, b):
    a, b = a.ravel(), b.ravel()
    pairs = np.unique(np.stack([a, b], 1), axis=0)
    return len(pairs) == len(np.unique(a)) == len(np.unique(b))


@pytest.mark.parametrize("N,Nc", [(2, 1), (4, 2), (5, 2), (7, 3), (3, 1)])
@pytest.mark.parametrize("periodic,dirichlet", [((False, False, False), "all"),
                                                ((True, True, False), "z"),
                                                ((True, False, True), "none")])
def test_coarse_mesh_equals_the_mesh_built_at_the_coarse_order(N, Nc, periodic, dirichlet):
    shape, lengths = (3, 4, 3), (1.0, 1.3, 0.7)
    kw = dict(periodic=periodic, dirichlet=dirichlet, jitter=0.08)
    fine = box_mesh(N, shape, lengths, **kw)
    ref = box_mesh(Nc, shape, lengths, **kw)
    xyz_c, gid_c, dir_c = coarse_mesh(fine.xyz, fine.gid, fine.dirichlet, N, Nc)
    np.testing.assert_allclose(xyz_c, ref.xyz, atol=1e-13)
    assert _same_partition(gid_c, ref.gid)
    if ref.dirichlet is None:
        assert dir_c is None
    else:
        np.testing.assert_array_equal(dir_c, ref.dirichlet)


def test_coarse_partition_on_a_deformed_clustered_mesh():
    kw = dict(periodic=(True, True, False), dirichlet="z", z_ratio=5.0,
              deform=dict(a=0.15, seed=1, kind="periodic"))
    fine = box_mesh(7, (3, 3, 4), (2.0, 2.0, 1.0), **kw)
    ref = box_mesh(3, (3, 3, 4), (2.0, 2.0, 1.0), **kw)
    _, gid_c, dir_c = coarse_mesh(fine.xyz, fine.gid, fine.dirichlet, 7, 3)
    assert _same_partition(gid_c, ref.gid)
    np.testing.assert_array_equal(dir_c, ref.dirichlet)


def test_prolongation_reproduces_coarse_polynomials_on_an_affine_mesh():
    N, Nc = 6, 3
    m = box_mesh(N, (2, 3, 2), (1.0, 1.5, 0.8), dirichlet="none")
    pmg = PMG(m.xyz, m.gid, m.dirichlet, N, orders=[N, Nc], coarse="exact")
    f = lambda x: (1 + x[..., 0] - x[..., 0] ** 3) * (x[..., 1] ** 2 + 0.3) * (2 - x[..., 2] ** 3)
    fine, coarse = pmg.levels
    xyz_c, _, _ = coarse_mesh(m.xyz, m.gid, None, N, Nc)
    fc = coarse.num.from_local_consistent(f(xyz_c))
    ff = fine.num.from_local_consistent(f(m.xyz))
    np.testing.assert_allclose(pmg.prolong(0, fc), ff, atol=1e-12)


def test_restriction_is_the_transpose_of_prolongation():
    m = box_mesh(5, (3, 2, 4), (1.0, 1.0, 1.0), periodic=(True, False, False), dirichlet="z",
                 jitter=0.05, z_ratio=3.0, deform=dict(a=0.1, seed=2, kind="walls"))
    pmg = PMG(m.xyz, m.gid, m.dirichlet, 5, coarse="exact")
    rng = np.random.default_rng(3)
    for l in range(len(pmg.levels) - 1):
        uc = rng.standard_normal(pmg.levels[l + 1].num.n_free)
        vf = rng.standard_normal(pmg.levels[l].num.n_free)
        a, b = pmg.prolong(l, uc) @ vf, uc @ pmg.restrict(l, vf)
        assert abs(a - b) <= 1e-13 * (np.abs(uc).sum() * np.abs(vf).sum())


@pytest.mark.parametrize("dirichlet", ["all", "none"])
def test_vcycle_with_exact_coarse_solve_is_symmetric_positive(dirichlet):
    m = box_mesh(5, (2, 3, 4), (1.0, 1.0, 1.0), dirichlet=dirichlet, jitter=0.05,
                 z_ratio=3.0, deform=dict(a=0.1, seed=2, kind="walls"))
    pmg = PMG(m.xyz, m.gid, m.dirichlet, 5, coarse="exact")
    n = pmg.levels[0].num.n_free
    rng = np.random.default_rng(4)
    for _ in range(3):
        r, s = rng.standard_normal(n), rng.standard_normal(n)
        if dirichlet == "none":  # the V-cycle acts on the mean-free subspace
            r, s = r - r.mean(), s - s.mean()
        Vr, Vs = pmg.vcycle(r), pmg.vcycle(s)
        if dirichlet == "none":
            Vr, Vs = Vr - Vr.mean(), Vs - Vs.mean()
        assert abs(Vr @ s - r @ Vs) <= 1e-11 * np.linalg.norm(Vr) * np.linalg.norm(s)
        assert Vr @ r > 0


@pytest.mark.parametrize("cfg,N", [(1, 7), (3, 9)])
def test_pmg_fcg_converges_fast_to_the_jacobi_pcg_solution(cfg, N):
    m, fld = config_mesh(cfg, N=N)
    pmg = PMG(m.xyz, m.gid, m.dirichlet, N)
    P = pmg.levels[0]
    b = P.rhs_from_source(fld["f"] * 3 * np.pi ** 2)
    ref = P.solve(b, rtol=1e-12)
    res = pmg.solve(b, rtol=1e-10)
    assert res["converged"]
    assert res["iters"] <= 0.15 * ref["iters"], (res["iters"], ref["iters"])
    err = np.linalg.norm(res["x"] - ref["x"]) / np.linalg.norm(ref["x"])
    assert err <= 1e-8, err


def test_pmg_fcg_neumann_box():
    m = box_mesh(5, (3, 3, 4), (1.0, 1.0, 1.0), dirichlet="none", z_ratio=5.0,
                 deform=dict(a=0.15, seed=1, kind="walls"))
    pmg = PMG(m.xyz, m.gid, m.dirichlet, 5)
    P = pmg.levels[0]
    b = np.random.default_rng(5).standard_normal(P.num.n_free)
    b -= b.mean()
    res = pmg.solve(b, rtol=1e-10)
    ref = P.solve(b, rtol=1e-12)
    assert res["converged"] and res["iters"] <= 0.2 * ref["iters"], (res["iters"], ref["iters"])
    assert abs(res["x"].mean()) <= 1e-12 * np.abs(res["x"]).max()
    assert np.linalg.norm(res["x"] - ref["x"]) <= 1e-8 * np.linalg.norm(ref["x"])

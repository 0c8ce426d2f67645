"""Edge cases of the solve paths on the GPU, against the oracle.

* One element: no node has several copies, so the in-solve operator's shared
  range, the segmented sums and sem_gs are empty.
* No unknowns: every node Dirichlet (one order-1 element), where every entry
  point must return zeros rather than fail inside a preconditioner set-up.
* The highest order, N = 10, through Jacobi PCG, the Chebyshev pass inside the
  CG (FP64 against the oracle's flexible CG, FP32 to 1e-10) and the
  p-multigrid preconditioner.
Tolerances: operator 1e-12, solution x 1e-8 against the oracle's solve at
1e-12, true residual by the oracle's operator 1.2e-10.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle.operator import local_apply
from sem_inputs import box_mesh, config_mesh

pytestmark = pytest.mark.gpu

sem = pytest.importorskip("paper_2501_13240_amd")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def one_element(N, dirichlet):
    return box_mesh(N, (1, 1, 1), (1.0, 1.3, 0.8), dirichlet=dirichlet, jitter=0.0,
                    deform=dict(a=0.1, seed=5, kind="walls"))


def _check_solve(M, P, bL, b_or, **kw):
    x, st = sem.solve(M, bL, rtol=1e-10, **kw)
    xf = P.num.from_local_consistent(x.cpu().numpy())
    r = P.project(b_or) - P.apply(xf)
    res = np.linalg.norm(r) / np.linalg.norm(P.project(b_or))
    ref = P.solve(b_or, rtol=1e-12)
    print(f"  {kw}: {st['iters']} it, true rel res {res:.2e}, x vs oracle {rel(xf, ref['x']):.2e}")
    assert st["converged"] == 1 and res <= 1.2e-10
    assert rel(xf, ref["x"]) <= 1e-8


@pytest.mark.parametrize("N", [2, 5, 7, 10])
def test_one_element_dirichlet(N):
    m = one_element(N, "all")
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    assert M.info["n_shared"] == 0 and M.info["n_free"] == (N - 1) ** 3
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, N)
    u = np.random.default_rng(N).standard_normal((1, (N + 1) ** 3))
    w = sem.ax(M, dev(u)).cpu().numpy()
    assert rel(w, local_apply(u, P.G, P.B, N)) <= 1e-12
    v = dev(u)
    assert torch.equal(sem.gs(M, v.clone()), v)  # no node has two copies
    b_or = P.rhs_from_source(np.ones((1, (N + 1) ** 3)))
    bL = sem.gs(M, sem.mass(M, torch.ones(1, (N + 1) ** 3, dtype=torch.float64,
                                          device="cuda")))
    _check_solve(M, P, bL, b_or)
    _check_solve(M, P, bL, b_or, precond="chebyshev", precond_prec="fp64")
    _check_solve(M, P, bL, b_or, precond="chebyshev", precond_prec="fp32")
    M.close()


@pytest.mark.parametrize("N", [5, 7])
def test_one_element_neumann(N):
    m = one_element(N, "none")
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    assert M.info["has_nullspace"] == 1 and M.info["n_shared"] == 0
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, N)
    rng = np.random.default_rng(3)
    bf = rng.standard_normal(P.num.n_free)
    bf -= bf.mean()
    bL = dev(P.num.to_local(bf))
    _check_solve(M, P, bL, bf)
    _check_solve(M, P, bL, bf, precond="chebyshev", precond_prec="fp32")
    _check_solve(M, P, bL, bf, mode="mixed_ir", precond="chebyshev", precond_prec="fp32")
    M.close()


def test_no_unknowns_return_zeros():
    m = box_mesh(1, (1, 1, 1), dirichlet="all")
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, 1)
    assert M.info["n_free"] == 0
    b = torch.ones(1, 8, dtype=torch.float64, device="cuda")
    for kw in (dict(), dict(precond="chebyshev", precond_prec="fp32"),
               dict(mode="mixed_ir", precond="jacobi", precond_prec="fp32")):
        x, st = sem.solve(M, b, x0=torch.full_like(b, 5.0), **kw)
        assert st["converged"] == 1 and st["iters"] == 0, kw
        assert bool((x == 0).all()), kw
    assert bool((sem.jacobi_inverse(M) == 0).all())
    assert bool((sem.cheb_apply(M, b, 2.0) == 0).all())
    assert bool((sem.cheb_apply_noalloc(M, b, 2.0, prec="fp32") == 0).all())
    with pytest.raises(sem.SemError, match="no free node"):
        sem.lmax_estimate(M)
    kb, bb, _ = sem.solve_backward(M, torch.zeros_like(b), b)
    assert bool((kb == 0).all()) and bool((bb == 0).all())
    M.close()


def test_order_10_solves_match_oracle():
    m, fld = config_mesh(1, N=10, shape=(2, 3, 2))
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N)
    f = fld["f"] * 3 * np.pi ** 2
    b_or = P.rhs_from_source(f)
    bL = sem.gs(M, sem.mass(M, dev(f)))
    _check_solve(M, P, bL, b_or)
    _check_solve(M, P, bL, b_or, precond="chebyshev", precond_prec="fp32")
    M.setup_pmg()
    _check_solve(M, P, bL, b_or, precond="pmg", precond_prec="fp32")
    lmax = 1.1 * sem.lmax_estimate(M)
    ref = P.solve(b_or, rtol=1e-30, max_iter=20, precond="chebyshev", m=3, rho_hat=lmax,
                  fixed_iters=True)
    x, st = sem.solve(M, bL, precond="chebyshev", precond_prec="fp64", lmax=lmax,
                      max_iter=20, fixed_iters=True, history=True)
    np.testing.assert_allclose(st["history"], ref["res_hist"], rtol=1e-8)
    M.close()

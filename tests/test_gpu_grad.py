"""Gradients of the differentiable solve x = A(k)^{-1} b on the GPU.

Variable-coefficient Helmholtz -div(k grad u) + h2 u, k = exp(0.5 g) with g a
smooth seeded random field, h2 = 1, Dirichlet walls; loss
L = sum over free unique nodes of (x - x_target)^2 with x_target the
continuous solution for k = 1.

* small instance of the recipe: autograd gradients for k and b against the
  oracle's adjoint gradient (1e-9 relative);
* full 16^3, N = 7 instance: 20 central finite differences in random k
  directions (relative 1e-6, eps = 1e-4, solves at 1e-13).
"""

import numpy as np
import pytest
import torch

import oracle
from sem_inputs import config_mesh

pytestmark = pytest.mark.gpu

sem = pytest.importorskip("paper_2501_13240_amd")


def _setup(shape=None, N=None):
    m, fld = config_mesh(4, N=N, shape=shape)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    h2 = fld["h2"]
    k = torch.tensor(fld["k"], device="cuda")
    f = torch.tensor(fld["f"], device="cuda")
    b = sem.gs(M, sem.mass(M, f))
    target = (f / (3 * np.pi ** 2 + h2)).contiguous()
    return m, fld, M, k, b, target, h2


def _loss(M, x, target):
    # sum over unique free nodes: local copies weighted by 1/multiplicity
    d = sem.mask(M, (x - target).contiguous())
    return torch.sum(d * d / M.multiplicity())


@pytest.mark.parametrize("precond", ["jacobi", "pmg"])
def test_autograd_matches_oracle_adjoint_gradient(precond):
    # the forward and the adjoint solve take the same options: Jacobi PCG, or
    # FP64 flexible CG with the FP32 p-multigrid cycle (k on every level)
    m, fld, M, k, b, target, h2 = _setup(shape=(4, 4, 4), N=5)
    opts = {}
    if precond == "pmg":
        M.setup_pmg()
        opts = dict(precond="pmg", precond_prec="fp32")
    kk = k.clone().requires_grad_(True)
    bb = b.clone().requires_grad_(True)
    x = sem.sem_solve(M, bb, k=kk, h2=h2, rtol=1e-13, **opts)
    L = _loss(M, x, target)
    L.backward()
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N, k=fld["k"], h2=h2)
    b_or = P.rhs_from_source(fld["f"])
    t_or = P.num.from_local_consistent(fld["f"]) / (3 * np.pi ** 2 + h2)
    g = oracle.solve_and_adjoint_gradient(P, b_or, t_or, rtol=1e-14)
    kbar = kk.grad.cpu().numpy()
    e_k = np.linalg.norm(kbar - g["kbar_local"]) / np.linalg.norm(g["kbar_local"])
    # b is read as the mean of its copies: dL/db_L = lambda / multiplicity
    lam_L = P.num.to_local(g["lam"])
    e_b = np.linalg.norm(bb.grad.cpu().numpy() - lam_L / P.num.mult[P.num.lid]) / np.linalg.norm(
        lam_L / P.num.mult[P.num.lid])
    print(f"gradient vs oracle adjoint: k {e_k:.2e}, b {e_b:.2e}; loss {float(L):.6e} vs {g['L']:.6e}")
    assert abs(float(L) - g["L"]) <= 1e-9 * g["L"]
    assert e_k <= 1e-9 and e_b <= 1e-9


def test_gradient_in_k_matches_20_central_differences_full_size():
    m, fld, M, k, b, target, h2 = _setup()
    kk = k.clone().requires_grad_(True)
    x = sem.sem_solve(M, b, k=kk, h2=h2, rtol=1e-13)
    L = _loss(M, x, target)
    L.backward()
    kbar = kk.grad.detach()
    gen = np.random.default_rng(5)
    eps = 1e-4
    worst = 0.0
    for i in range(20):
        dk = k * torch.tensor(gen.standard_normal(k.shape), device="cuda")
        with torch.no_grad():
            xp, _ = sem.solve(M, b, k=(k + eps * dk).contiguous(), h2=h2, rtol=1e-13, max_iter=50000)
            xm, _ = sem.solve(M, b, k=(k - eps * dk).contiguous(), h2=h2, rtol=1e-13, max_iter=50000)
            fd = (float(_loss(M, xp, target)) - float(_loss(M, xm, target))) / (2 * eps)
        ad = float(torch.sum(kbar * dk))
        err = abs(fd - ad) / abs(fd)
        worst = max(worst, err)
        assert err <= 1e-6, (i, fd, ad, err)
    print(f"20 central differences: worst relative error {worst:.2e}")


def test_ax_backward_dot_product_identities():
    m, fld, M, k, b, target, h2 = _setup(shape=(6, 5, 4))
    g = torch.Generator(device="cuda").manual_seed(3)
    u = torch.randn(M.E, M.P, dtype=torch.float64, device="cuda", generator=g)
    wb = torch.randn(M.E, M.P, dtype=torch.float64, device="cuda", generator=g)
    dk = torch.randn(M.E, M.P, dtype=torch.float64, device="cuda", generator=g)
    ub, kb = sem.ax_backward(M, u, wb, k=k, h2=h2)
    lhs = float(torch.sum(wb * sem.ax(M, u, k=dk)))
    rhs = float(torch.sum(dk * kb))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    a = float(torch.sum(wb * sem.ax(M, u, k=k, h2=h2)))
    c = float(torch.sum(u * ub))
    assert abs(a - c) <= 1e-12 * abs(a)


@pytest.mark.parametrize("case", ["helmholtz_k", "neumann"])
def test_solve_backward_matches_oracle_adjoint(case):
    """sem_solve_backward through the C ABI for an arbitrary cotangent xbar
    (not copy-consistent): the oracle's adjoint solve A lam = R Q^T xbar, then
    dL/dk = -kbar(lam_L, x_L) and dL/db = lam_L / multiplicity."""
    if case == "helmholtz_k":
        m, fld = config_mesh(4, N=5, shape=(4, 4, 3))
        k_np, h2 = fld["k"], fld["h2"]
        P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N, k=k_np, h2=h2)
        b_or = P.rhs_from_source(fld["f"])
    else:  # all-Neumann, constant mode removed, k = 1
        m, fld = config_mesh(5, N=7, shape=(3, 3, 3))
        k_np, h2 = None, 0.0
        P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N)
        b_or = P.num.from_local_consistent(fld["b"])
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    kd = None if k_np is None else torch.tensor(k_np, device="cuda")
    x_or = P.solve(b_or, rtol=1e-14)["x"]
    xbar = np.random.default_rng(8).standard_normal((m.E, m.P))
    lam = P.solve(P.num.R(P.num.Qt(xbar)), rtol=1e-14)["x"]
    kbar_or = -oracle.kgrad_contraction(P.num.to_local(x_or), P.num.to_local(lam), P.G, m.N)
    mult = P.num.mult[P.num.lid]
    bbar_or = P.num.to_local(lam) / mult
    x = torch.tensor(P.num.to_local(x_or), device="cuda")
    kbar, bbar, st = sem.solve_backward(M, x, torch.tensor(xbar, device="cuda"), k=kd, h2=h2,
                                        rtol=1e-14, max_iter=20000)
    e_k = np.linalg.norm(kbar.cpu().numpy() - kbar_or) / np.linalg.norm(kbar_or)
    e_b = np.linalg.norm(bbar.cpu().numpy() - bbar_or) / np.linalg.norm(bbar_or)
    print(f"{case}: adjoint solve {st['iters']} it; kbar {e_k:.2e}, bbar {e_b:.2e}")
    assert st["converged"] == 1
    assert e_k <= 1e-9 and e_b <= 1e-9
    # one output at a time gives the same values
    kb1, none_b, _ = sem.solve_backward(M, x, torch.tensor(xbar, device="cuda"), k=kd, h2=h2,
                                        need_bbar=False, rtol=1e-14, max_iter=20000)
    assert none_b is None and torch.equal(kb1, kbar)

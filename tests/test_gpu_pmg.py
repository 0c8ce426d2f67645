"""GPU parity of the p-multigrid preconditioner against the oracle.

The GPU's per-level Chebyshev bounds come from its own Lanczos runs (started
from a different vector than the oracle's), so V-cycle parity hands the GPU's
bounds to the oracle; the bounds themselves are checked against the oracle's
estimates and the dense generalised eigenvalue on a small mesh.

Tolerances:
  one V-cycle, FP64 arithmetic           <= 1e-9 relative (30 coarse CG
      iterations amplify rounding differences mildly)
  one V-cycle, FP32 arithmetic           <= 2e-4 relative
  solves: true FP64 residual <= 1e-10 (refinement: 1.2e-10), x within 1e-8 of
      the oracle's FP64 solution, iteration counts within 2 of the oracle's
"""

import numpy as np
import pytest
import torch

import oracle
from oracle.pmg import PMG, level_orders
from sem_inputs import box_mesh, config_mesh

pytestmark = pytest.mark.gpu

sem = pytest.importorskip("paper_2501_13240_amd")


# cycle parameters, passed explicitly to the library and to the oracle
_CYCLE = {"jacobi": dict(smooth_order=5, coarse_iters=20),
          "schwarz": dict(smooth_order=4, coarse_iters=30)}


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _vcycle_case(m, N, k=None, h2=0.0, seed=1, smoother="jacobi"):
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    M.setup_pmg(smoother=smoother, **_CYCLE[smoother])
    orders, _ = M.pmg_info()
    assert orders == level_orders(N)
    kd = None if k is None else dev(k)
    P0 = oracle.Problem(m.xyz, m.gid, m.dirichlet, N, k=k, h2=h2)
    rf = np.random.default_rng(seed).standard_normal(P0.num.n_free)
    if P0.neumann:
        rf -= rf.mean()
    rL = dev(P0.num.to_local(rf))
    z64 = sem.pmg_apply(M, rL, k=kd, h2=h2, prec="fp64").cpu().numpy()
    _, rho = M.pmg_info()
    z32 = sem.pmg_apply(M, rL, k=kd, h2=h2, prec="fp32").cpu().numpy()
    pmg = PMG(m.xyz, m.gid, m.dirichlet, N, k=k, h2=h2, rho=rho, smoother=smoother,
              **_CYCLE[smoother])
    z_or = P0.num.to_local(pmg.vcycle(rf))
    if P0.neumann:  # the cycle's output is defined up to a constant on a singular level
        mean = lambda zl: P0.num.from_local_consistent(zl).mean()
        z64, z32, z_or = z64 - mean(z64), z32 - mean(z32), z_or - mean(z_or)
    e64, e32 = rel(z64, z_or), rel(z32, z_or)
    print(f"N={N} {smoother} levels {orders} rho {np.round(rho, 3)}: V-cycle fp64 {e64:.2e}, "
          f"fp32 {e32:.2e}")
    # FP64: the same arithmetic in another order (measured 2e-15 .. 2e-14)
    assert e64 <= 1e-12
    assert e32 <= 2e-4
    return M, pmg, rho


def test_vcycle_matches_oracle_dirichlet_cube():
    m, _ = config_mesh(1, N=7)
    _vcycle_case(m, 7)


def test_vcycle_matches_oracle_neumann_clustered_box():
    m, _ = config_mesh(5, shape=(4, 4, 4))
    _vcycle_case(m, 9, seed=2)


def test_vcycle_matches_oracle_variable_k_helmholtz():
    m, fld = config_mesh(4, shape=(4, 4, 4))
    _vcycle_case(m, 7, k=fld["k"], h2=fld["h2"], seed=3)


def test_vcycle_periodic_deformed_box_ragged_orders():
    m = box_mesh(6, (5, 3, 4), (2.0, 1.0, 1.0), periodic=(True, True, False), dirichlet="z",
                 z_ratio=4.0, deform=dict(a=0.15, seed=1, kind="periodic"))
    _vcycle_case(m, 6, seed=4)


def test_level_bounds_bracket_the_largest_eigenvalue():
    m = box_mesh(4, (3, 3, 3), (1.0, 1.5, 1.0), dirichlet="all", jitter=0.05,
                 deform=dict(a=0.15, seed=3, kind="walls"))
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, 4)
    M.setup_pmg(smoother="jacobi", **_CYCLE["jacobi"])
    rL = dev(np.zeros((m.E, m.P)))
    sem.pmg_apply(M, rL)
    orders, rho = M.pmg_info()
    pmg = PMG(m.xyz, m.gid, m.dirichlet, 4, coarse="exact", smoother="jacobi")
    import scipy.linalg as sla
    for l, P in enumerate(pmg.levels):
        A = oracle.explicit_matrix(P.G, P.B, P.N, P.num).toarray()
        true = sla.eigh(A, np.diag(np.diag(A)), eigvals_only=True)[-1]
        est = rho[l] / 1.1
        print(f"level {l} (N={orders[l]}): estimate {est:.4f}, true {true:.4f}")
        assert 0.95 * true <= est <= true * (1 + 1e-10)


def _true_rel_residual(P, x_local, b_free):
    xf = P.num.from_local_consistent(x_local)
    if P.neumann:
        b_free = b_free - b_free.mean()
    return np.linalg.norm(b_free - P.apply(xf)) / np.linalg.norm(b_free), xf


@pytest.mark.parametrize("cfg,N", [(1, 7), (3, 9)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_pmg_fcg_matches_oracle(cfg, N, prec):
    m, fld = config_mesh(cfg, N=N)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    M.setup_pmg(smoother="jacobi", **_CYCLE["jacobi"])
    f = fld["f"] * 3 * np.pi ** 2
    bL = sem.gs(M, sem.mass(M, dev(f)))
    x, st = sem.solve(M, bL, precond="pmg", precond_prec=prec, rtol=1e-10)
    _, rho = M.pmg_info()
    pmg = PMG(m.xyz, m.gid, m.dirichlet, N, rho=rho, smoother="jacobi", **_CYCLE["jacobi"])
    P = pmg.levels[0]
    b_or = P.rhs_from_source(f)
    ref = pmg.solve(b_or, rtol=1e-10)
    jac = P.solve(b_or, rtol=1e-12)
    res, xf = _true_rel_residual(P, x.cpu().numpy(), b_or)
    print(f"cfg{cfg} N={N} pMG {prec}: iters gpu {st['iters']} oracle {ref['iters']} "
          f"(Jacobi {jac['iters']}), true rel res {res:.2e}, err {rel(xf, jac['x']):.2e}")
    assert st["converged"] == 1 and res <= 1e-10
    assert abs(st["iters"] - ref["iters"]) <= 2
    assert rel(xf, jac["x"]) <= 1e-8


def test_pmg_inside_mixed_refinement():
    m, fld = config_mesh(1, N=7)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, 7)
    f = fld["f"] * 3 * np.pi ** 2
    bL = sem.gs(M, sem.mass(M, dev(f)))
    x, st = sem.solve(M, bL, mode="mixed_ir", precond="pmg", rtol=1e-10)
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, 7)
    b_or = P.rhs_from_source(f)
    res, xf = _true_rel_residual(P, x.cpu().numpy(), b_or)
    print(f"mixed + pMG: outer {st['outer_iters']} inner {st['iters']} true rel res {res:.2e}")
    assert st["converged"] == 1 and res <= 1.2e-10


def test_pmg_fcg_neumann_clustered_box():
    m, fld = config_mesh(5, shape=(4, 4, 4))
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    M.setup_pmg(smoother="jacobi", **_CYCLE["jacobi"])
    b = dev(fld["b"])
    x, st = sem.solve(M, b, precond="pmg", rtol=1e-10)
    _, rho = M.pmg_info()
    pmg = PMG(m.xyz, m.gid, m.dirichlet, m.N, rho=rho, smoother="jacobi", **_CYCLE["jacobi"])
    P = pmg.levels[0]
    b_or = P.num.from_local_consistent(fld["b"])
    ref = pmg.solve(b_or, rtol=1e-10)
    res, xf = _true_rel_residual(P, x.cpu().numpy(), b_or)
    print(f"neumann pMG: iters gpu {st['iters']} oracle {ref['iters']}, res {res:.2e}")
    assert st["converged"] == 1 and res <= 1.05e-10
    assert abs(st["iters"] - ref["iters"]) <= 2
    assert abs(xf.mean()) <= 1e-10 * np.abs(xf).max()
    assert rel(xf, ref["x"]) <= 1e-7


def test_pmg_graph_replay_matches_eager():
    m, fld = config_mesh(1, N=5)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    M.setup_pmg(smoother="jacobi", **_CYCLE["jacobi"])
    b = sem.gs(M, sem.mass(M, dev(fld["f"])))
    x_e, st_e = sem.solve(M, b, precond="pmg", rtol=1e-10, profile=True)
    for rep in range(3):
        x_g, st_g = sem.solve(M, b, precond="pmg", rtol=1e-10)
        assert st_g["iters"] == st_e["iters"]
        assert torch.equal(x_g, x_e), rep
        sem.ax(M, x_g)
        torch.cuda.synchronize()


@pytest.fixture(scope="module")
def convection_box():
    """The 32x32x16, N = 7 convection box at full size with the oracle's
    assembled problem on it (the true residual of the GPU solutions)."""
    m, fld = config_mesh(2)
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N)
    return m, fld, P


def _oracle_true_res(P, x, b_local):
    b = P.num.from_local_consistent(b_local)
    xf = P.num.from_local_consistent(x.cpu().numpy())
    return np.linalg.norm(b - P.apply(xf)) / np.linalg.norm(b)


@pytest.mark.timeout(900)
def test_pmg_full_convection_box_converges(convection_box):
    """Jacobi-smoothed p-multigrid on the full convection box: flexible CG
    with the FP32 and the FP64 cycle to 1e-10, the oracle's operator giving
    the true residual, in a small fraction of the Jacobi-PCG iterations."""
    m, fld, P = convection_box
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    M.setup_pmg(smoother="jacobi", **_CYCLE["jacobi"])
    b = dev(fld["b"])
    for prec in ("fp32", "fp64"):
        x, st = sem.solve(M, b, precond="pmg", precond_prec=prec, rtol=1e-10)
        res = _oracle_true_res(P, x, fld["b"])
        print(f"convection box pMG ({prec} cycle): {st['iters']} iterations, "
              f"{st['time_ms']:.1f} ms, oracle true res {res:.2e}")
        assert st["converged"] == 1 and res <= 1.2e-10
        assert st["iters"] <= 80
    M.close()


def test_pmg_errors():
    import ctypes
    from paper_2501_13240_amd import _lib as L
    m, fld = config_mesh(1, N=3)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    b = dev(fld["f"])
    z = torch.empty_like(b)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # no hierarchy yet
    assert M._lib.sem_pmg_apply(M.handle, ctypes.c_void_p(b.data_ptr()),
                                ctypes.c_void_p(z.data_ptr()), None, 0.0, 1, stream) == L.SEM_EINVAL
    for bad in (dict(orders=[3, 3, 1]), dict(orders=[2, 1]), dict(smooth_order=0),
                dict(coarse_iters=0)):
        with pytest.raises(sem.SemError, match="EINVAL"):
            M.setup_pmg(**bad)
    with pytest.raises(sem.SemError, match="EINVAL"):
        sem.solve(M, b, mode="mixed_ir", precond="pmg", precond_prec="fp64")


# ------------------------------------------------------------ Schwarz smoothing

def test_schwarz_vcycle_matches_oracle_dirichlet_cube():
    m, _ = config_mesh(1, N=7)
    _vcycle_case(m, 7, smoother="schwarz")


def test_schwarz_vcycle_matches_oracle_neumann_clustered_box(store_form):
    # the order-9 level forms its smoother residuals with the split operator,
    # in both store forms
    m, _ = config_mesh(5, shape=(4, 4, 4))
    _vcycle_case(m, 9, seed=2, smoother="schwarz")


def test_schwarz_vcycle_periodic_deformed_box_variable_k():
    m = box_mesh(6, (5, 3, 4), (2.0, 1.0, 1.0), periodic=(True, True, False), dirichlet="z",
                 z_ratio=4.0, deform=dict(a=0.15, seed=1, kind="periodic"))
    k = np.exp(0.3 * np.random.default_rng(9).standard_normal((m.E, m.P)))
    _vcycle_case(m, 6, k=k, h2=0.5, seed=4, smoother="schwarz")


def test_schwarz_bound_brackets_the_largest_eigenvalue():
    """lambda_max of the Schwarz-preconditioned operator on each smoothing
    level: the GPU's 20-step Lanczos estimate against a dense eigensolver."""
    m = box_mesh(4, (3, 3, 3), (1.0, 1.5, 1.0), dirichlet="all", jitter=0.05,
                 deform=dict(a=0.15, seed=3, kind="walls"))
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, 4)
    M.setup_pmg(smoother="schwarz")
    sem.pmg_apply(M, dev(np.zeros((m.E, m.P))))
    orders, rho = M.pmg_info()
    pmg = PMG(m.xyz, m.gid, m.dirichlet, 4, coarse="exact", smoother="schwarz")
    for l in range(len(orders) - 1):
        P = pmg.levels[l]
        A = oracle.explicit_matrix(P.G, P.B, P.N, P.num).toarray()
        n = A.shape[0]
        Smat = np.stack([pmg.S[l](np.eye(n)[i]) for i in range(n)], 1)
        true = np.max(np.linalg.eigvals(Smat @ A).real)
        est = rho[l] / 1.1
        print(f"level {l} (N={orders[l]}): Schwarz bound {est:.4f}, true {true:.4f}")
        assert 0.95 * true <= est <= true * (1 + 1e-8)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_schwarz_pmg_fcg_matches_oracle(prec, store_form):
    m, fld = config_mesh(3, N=9)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, 9)
    M.setup_pmg(smoother="schwarz", **_CYCLE["schwarz"])
    f = fld["f"] * 3 * np.pi ** 2
    bL = sem.gs(M, sem.mass(M, dev(f)))
    x, st = sem.solve(M, bL, precond="pmg", precond_prec=prec, rtol=1e-10)
    _, rho = M.pmg_info()
    pmg = PMG(m.xyz, m.gid, m.dirichlet, 9, rho=rho, smoother="schwarz", **_CYCLE["schwarz"])
    P = pmg.levels[0]
    b_or = P.rhs_from_source(f)
    ref = pmg.solve(b_or, rtol=1e-10)
    jac = P.solve(b_or, rtol=1e-12)
    res, xf = _true_rel_residual(P, x.cpu().numpy(), b_or)
    print(f"Schwarz pMG {prec}: iters gpu {st['iters']} oracle {ref['iters']}, res {res:.2e}")
    assert st["converged"] == 1 and res <= 1e-10
    assert abs(st["iters"] - ref["iters"]) <= 2
    assert rel(xf, jac["x"]) <= 1e-8


def test_schwarz_pmg_neumann_and_refinement():
    m, fld = config_mesh(5, shape=(4, 4, 4))
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    M.setup_pmg(smoother="schwarz")
    b = dev(fld["b"])
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N)
    b_or = P.num.from_local_consistent(fld["b"])
    for mode in ("cg", "mixed_ir"):
        x, st = sem.solve(M, b, mode=mode, precond="pmg", rtol=1e-10)
        res, xf = _true_rel_residual(P, x.cpu().numpy(), b_or)
        print(f"Schwarz pMG neumann {mode}: iters {st['iters']} outer {st['outer_iters']} "
              f"res {res:.2e}")
        assert st["converged"] == 1 and res <= 1.2e-10


def test_schwarz_pmg_graph_replay_matches_eager():
    m, fld = config_mesh(1, N=5)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    M.setup_pmg(smoother="schwarz")
    b = sem.gs(M, sem.mass(M, dev(fld["f"])))
    x_e, st_e = sem.solve(M, b, precond="pmg", rtol=1e-10, profile=True)
    for rep in range(3):
        x_g, st_g = sem.solve(M, b, precond="pmg", rtol=1e-10)
        assert st_g["iters"] == st_e["iters"]
        assert torch.equal(x_g, x_e), rep
        sem.ax(M, x_g)
        torch.cuda.synchronize()


@pytest.mark.timeout(900)
def test_schwarz_pmg_full_convection_box(convection_box):
    """The default (Schwarz-smoothed) p-multigrid on the full convection box,
    FP32 and FP64 cycles, to 1e-10 by the oracle's true residual."""
    m, fld, P = convection_box
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    M.setup_pmg(smoother="schwarz")
    b = dev(fld["b"])
    for prec in ("fp32", "fp64"):
        x, st = sem.solve(M, b, precond="pmg", precond_prec=prec, rtol=1e-10)
        res = _oracle_true_res(P, x, fld["b"])
        print(f"convection box Schwarz pMG ({prec} cycle): {st['iters']} iterations, "
              f"{st['time_ms']:.1f} ms, oracle true res {res:.2e}")
        assert st["converged"] == 1 and res <= 1.2e-10
        assert st["iters"] <= 20
    M.close()

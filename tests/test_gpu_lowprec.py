"""GPU parity of the 16-bit contraction operator (bfloat16 / IEEE half
operands on the matrix cores, FP32 accumulation) against the oracle's
emulation of the same roundings, and of the solves that use it as the
Chebyshev preconditioner's operator.

Tolerances:
  operator vs the oracle's emulation  <= 3e-5 relative (2-norm); the rest is
      FP32 arithmetic and the rare operand that lands on the other side of a
      16-bit rounding midpoint because its FP32 value differs in the last bits
  operator vs the exact FP64 operator <= 4.2 u |D|^T|G||D||u| per point
      (the a-priori rounding bound, u = 2^-8 bf16, 2^-11 half)
  Chebyshev apply vs the oracle's     <= 1e-4 relative
  solves: true FP64 residual <= 1e-10 (mixed: 1.2e-10), x within 1e-7 of the
      oracle's FP64 solution
"""

import numpy as np
import pytest
import torch

import oracle
from oracle.geometry import geometric_factors
from oracle.operator import local_apply, local_apply_lowprec, local_apply_majorant
from sem_inputs import box_mesh, config_mesh, random_local_normal

pytestmark = pytest.mark.gpu

sem = pytest.importorskip("paper_2501_13240_amd")

UNIT = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}


def rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300)


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def small_mesh(N, shape=(3, 2, 3)):
    return box_mesh(N, shape, (1.0, 1.5, 1.0), dirichlet="all", jitter=0.05,
                    deform=dict(a=0.15, seed=3, kind="walls"))


def _check_apply(w, u, G, B, N, fmt, k, h2, scale_tag=""):
    w_em = local_apply_lowprec(u, G, B, N, fmt, k=k, h2=h2)
    w_ex = local_apply(u, G, B, N, k=k, h2=h2)
    bound = (np.abs(w - w_ex) / (UNIT[fmt] * local_apply_majorant(u, G, N, k=k))).max()
    e_em, e_ex = rel(w, w_em), rel(w, w_ex)
    print(f"N={N} {fmt}{scale_tag}: vs emulation {e_em:.2e}, vs exact {e_ex:.2e}, "
          f"bound ratio {bound:.2f}")
    assert e_em <= 3e-5
    assert bound <= 4.2


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
@pytest.mark.parametrize("N", [1, 2, 4, 5, 7, 9, 10])
@pytest.mark.parametrize("with_k", [False, True])
def test_ax_16bit_matches_oracle_emulation(fmt, N, with_k):
    m = small_mesh(N)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    Go, Bo, _ = geometric_factors(m.xyz, N)
    u = f32(random_local_normal((m.E, m.P), 300 + N))
    k = f32(np.exp(0.5 * random_local_normal((m.E, m.P), 400 + N))) if with_k else None
    h2 = 0.7 if with_k else 0.0
    w = sem.ax(M, dev(u, torch.float32), k=None if k is None else dev(k, torch.float32), h2=h2,
               prec=f"{fmt}_mfma").cpu().numpy().astype(np.float64)
    _check_apply(w, u, Go, Bo, N, fmt, k, h2)


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_ax_16bit_keeps_residual_sized_inputs(fmt):
    """Inputs far below half precision's normal range (a late residual)."""
    N = 7
    m = small_mesh(N)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    Go, Bo, _ = geometric_factors(m.xyz, N)
    u = f32(1e-9 * random_local_normal((m.E, m.P), 500))
    w = sem.ax(M, dev(u, torch.float32), prec=f"{fmt}_mfma").cpu().numpy().astype(np.float64)
    _check_apply(w, u, Go, Bo, N, fmt, None, 0.0, " x1e-9")


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_ax_16bit_full_convection_box_sampled_elements(fmt):
    """The 32x32x16, N=7 convection box at full size: the operator is
    element-local, so the oracle checks a seeded sample of 24 elements."""
    m, _ = config_mesh(2)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    u = f32(random_local_normal((m.E, m.P), 600))
    w = sem.ax(M, dev(u, torch.float32), prec=f"{fmt}_mfma").cpu().numpy().astype(np.float64)
    sel = np.sort(np.random.default_rng(601).choice(m.E, 24, replace=False))
    sel[-1] = m.E - 1
    Go, Bo, _ = geometric_factors(m.xyz[sel], m.N)
    _check_apply(w[sel], u[sel], Go, Bo, m.N, fmt, None, 0.0, " (sampled)")


def _lowprec_problem_apply(P, fmt):
    num = P.num

    def A(xf):
        uL = f32(num.to_local(xf))
        return num.R(num.Qt(local_apply_lowprec(uL, P.G, P.B, P.N, fmt, k=P.k, h2=P.h2)))
    return A


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_chebyshev_apply_16bit_matches_oracle(fmt):
    m, _ = config_mesh(1, N=5)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N)
    rf = np.random.default_rng(7).standard_normal(P.num.n_free)
    lmax = 2.3
    z_or = oracle.chebyshev_apply(_lowprec_problem_apply(P, fmt), 1.0 / P.diag(), rf, 3, lmax)
    z_ex = oracle.chebyshev_apply(P.apply, 1.0 / P.diag(), rf, 3, lmax)
    z = sem.cheb_apply(M, dev(P.num.to_local(rf)), lmax, order=3,
                       prec=f"{fmt}_mfma").cpu().numpy()
    e, e_ex = rel(z, P.num.to_local(z_or)), rel(z, P.num.to_local(z_ex))
    print(f"{fmt} Chebyshev: vs emulation {e:.2e}, vs exact-operator Chebyshev {e_ex:.2e}")
    assert e <= 1e-4


def _true_rel_residual(P, x_local, b_free):
    xf = P.num.from_local_consistent(x_local)
    return np.linalg.norm(b_free - P.apply(xf)) / np.linalg.norm(b_free), xf


@pytest.mark.parametrize("N", [7, 9])  # the precision workload at both orders
@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
@pytest.mark.parametrize("mode", ["cg", "mixed_ir"])
def test_solves_with_16bit_chebyshev_reach_fp64_tolerance(fmt, mode, N):
    m, fld = config_mesh(1, N=N)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N)
    f = fld["f"] * 3 * np.pi ** 2
    b_or = P.rhs_from_source(f)
    ref = P.solve(b_or, rtol=1e-12)
    bL = sem.gs(M, sem.mass(M, dev(f)))
    x, st = sem.solve(M, bL, mode=mode, precond="chebyshev", precond_prec=f"{fmt}_mfma",
                      rtol=1e-10)
    _, st32 = sem.solve(M, bL, mode=mode, precond="chebyshev", precond_prec="fp32", rtol=1e-10)
    res, xf = _true_rel_residual(P, x.cpu().numpy(), b_or)
    print(f"N={N} {mode} + {fmt} Chebyshev: iters {st['iters']} (fp32 Chebyshev {st32['iters']}), "
          f"outer {st['outer_iters']}, true rel res {res:.2e}, err vs oracle {rel(xf, ref['x']):.2e}")
    assert st["converged"] == 1
    assert res <= (1.0e-10 if mode == "cg" else 1.2e-10)
    assert rel(xf, ref["x"]) <= 1e-7

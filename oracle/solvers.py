"""O8-O12: the assembled problem, preconditioned CG, Chebyshev, Lanczos.

Test infrastructure only (see the package docstring).

The pressure Poisson solve is the stiffest substep of each time step and is
solved iteratively with a preconditioner (Sec. 2.2).  The Krylov method and the
Jacobi preconditioner are the textbook ones (the paper names neither):

PCG (Hestenes-Stiefel), x0 = 0 unless given, S = diag(A)^{-1}:
  r = b - A x, z = S r, p = z, rho = r.z
  repeat:  w = A p;  alpha = rho / p.w;  x += alpha p;  r -= alpha w;
           stop if ||r||_2 <= rtol ||b||_2;
           z = M^{-1} r;  beta = r.z / rho  (flexible: z.(r - r_old) / rho);
           rho = r.z;  p = z + beta p

Fourth-kind Chebyshev acceleration (Sec. 2.2) of the Jacobi iteration, as
given by Lottes (2022) for a bound rho_hat >= lambda_max(S A), zero start:
  d_0 = 4/(3 rho_hat) S r_0
  for k = 1..m-1:  x_k = x_{k-1} + d_{k-1};  r_k = r_{k-1} - A d_{k-1};
                   d_k = (2k-1)/(2k+3) d_{k-1} + (8k+4)/((2k+3) rho_hat) S r_k
  z = x_{m-1} + d_{m-1}
whose error polynomial is e_m(lambda) = W_m(1 - 2 lambda/rho_hat) / (2m+1),
W_m the fourth-kind Chebyshev polynomial (pinned in the tests).

Vectors here live on the free unique nodes (length n_free); dot products are
unique-node dot products.
"""

from __future__ import annotations

import numpy as np

from .assembly import Numbering
from .geometry import geometric_factors
from .operator import local_apply, local_diagonal


class Problem:
    """The assembled problem R Q^T A_L(k) Q R^T on one mesh."""

    def __init__(self, xyz, gid, dirichlet, N, k=None, h2=0.0):
        self.N = N
        self.num = Numbering(gid, dirichlet)
        self.G, self.B, self.detJ = geometric_factors(xyz, N)
        self.k = None if k is None else np.asarray(k, dtype=np.float64)
        self.h2 = float(h2)
        self.neumann = self.num.n_free == self.num.n and self.h2 == 0.0

    def set_k(self, k):
        self.k = None if k is None else np.asarray(k, dtype=np.float64)

    def apply_local(self, uL):
        return local_apply(uL, self.G, self.B, self.N, k=self.k, h2=self.h2)

    def apply(self, xf: np.ndarray) -> np.ndarray:
        num = self.num
        return num.R(num.Qt(self.apply_local(num.to_local(xf))))

    def diag(self) -> np.ndarray:
        d = local_diagonal(self.G, self.B, self.N, k=self.k, h2=self.h2)
        return self.num.R(self.num.Qt(d))

    def rhs_from_source(self, f: np.ndarray) -> np.ndarray:
        """b = R Q^T (B f): mass-weighted load vector of a pointwise source."""
        return self.num.R(self.num.Qt(self.B * f))

    def project(self, v: np.ndarray) -> np.ndarray:
        """Remove the constant (null-space) mode over the unique nodes."""
        return v - v.mean() if self.neumann else v

    def solve(self, b, rtol=1e-10, max_iter=10000, precond="jacobi", m=3, rho_hat=None,
              x0=None, fixed_iters=False):
        dinv = 1.0 / self.diag()
        proj = self.project if self.neumann else None
        if self.neumann:
            b = b - b.mean()
        if precond == "jacobi":
            M = lambda r: dinv * r
            flexible = False
        elif precond == "chebyshev":
            if rho_hat is None:
                rng = np.random.default_rng(7)
                rho_hat = 1.1 * lanczos_lmax(self.apply, dinv, rng.standard_normal(b.size), 20, proj)
            M = lambda r: chebyshev_apply(self.apply, dinv, r, m, rho_hat)
            flexible = True
        elif precond == "chebyshev1":
            if rho_hat is None:
                rng = np.random.default_rng(7)
                rho_hat = 1.1 * lanczos_lmax(self.apply, dinv, rng.standard_normal(b.size), 20, proj)
            M = lambda r: chebyshev1_apply(self.apply, dinv, r, m, rho_hat)
            flexible = True
        else:
            raise ValueError(precond)
        res = pcg(self.apply, b, M, rtol=rtol, max_iter=max_iter, x0=x0,
                  fixed_iters=fixed_iters, flexible=flexible, project=proj)
        if self.neumann:
            res["x"] = res["x"] - res["x"].mean()
        return res


def pcg(A, b, M, rtol=1e-10, max_iter=10000, x0=None, fixed_iters=False,
        flexible=False, project=None):
    """Preconditioned CG; returns dict(x, iters, res_hist, alpha, beta, converged)."""
    n = b.size
    x = np.zeros(n) if x0 is None else x0.astype(np.float64).copy()
    r = b - A(x) if x0 is not None else b.copy()
    if project is not None:
        r = project(r)
    bnorm = np.linalg.norm(b)
    hist = [np.linalg.norm(r)]
    alphas, betas = [], []
    if bnorm == 0.0:
        return dict(x=np.zeros(n), iters=0, res_hist=np.array(hist), alpha=np.array([]),
                    beta=np.array([]), converged=True)
    z = M(r)
    p = z.copy()
    rho = r @ z
    it = 0
    converged = False
    while it < max_iter:
        w = A(p)
        pw = p @ w
        if not (pw > 0.0):
            raise FloatingPointError("CG breakdown: p.Ap <= 0")
        alpha = rho / pw
        x = x + alpha * p
        r_old = r
        r = r - alpha * w
        if project is not None:
            r = project(r)
        it += 1
        alphas.append(alpha)
        hist.append(np.linalg.norm(r))
        if not fixed_iters and hist[-1] <= rtol * bnorm:
            converged = True
            break
        z_new = M(r)
        rho_new = r @ z_new
        beta = (z_new @ (r - r_old)) / rho if flexible else rho_new / rho
        betas.append(beta)
        p = z_new + beta * p
        rho = rho_new
    if fixed_iters:
        converged = hist[-1] <= rtol * bnorm
    return dict(x=x, iters=it, res_hist=np.array(hist), alpha=np.array(alphas),
                beta=np.array(betas), converged=converged)


def _as_operator(S):
    """The preconditioner S as a function: a callable, or a diagonal given as
    an array."""
    return S if callable(S) else (lambda v: S * v)


def chebyshev_apply(A, dinv, r, m, rho_hat):
    """z = p_m(S A) S r, fourth-kind Chebyshev of order m (m-1 operator
    applies); S is the Jacobi diagonal (array) or another symmetric
    preconditioner (callable, e.g. a Schwarz smoother)."""
    S = _as_operator(dinv)
    d = (4.0 / (3.0 * rho_hat)) * S(r)
    x = np.zeros_like(r)
    rk = r.copy()
    for k in range(1, m):
        x = x + d
        rk = rk - A(d)
        d = ((2 * k - 1) / (2 * k + 3)) * d + ((8 * k + 4) / ((2 * k + 3) * rho_hat)) * S(rk)
    return x + d


def chebyshev1_apply(A, dinv, r, m, rho_hat, ratio=10.0):
    """z = p_m(S A) S r, the classical (first-kind) Chebyshev semi-iteration
    of order m (m-1 operator applies) from zero on the interval
    [rho_hat / ratio, rho_hat]: with theta the interval's centre, delta its
    half width and sigma = theta / delta, the iterates follow the three-term
    recurrence of the scaled first-kind polynomials,
        d_0 = S r / theta,  x_1 = d_0,
        rho_0 = 1 / sigma,  rho_k = 1 / (2 sigma - rho_{k-1}),
        r_k = r_{k-1} - A d_{k-1},
        d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) S r_k,
        x_{k+1} = x_k + d_k,
    so that the error polynomial is 1 - lambda p(lambda) =
    T_m((theta - lambda) / delta) / T_m(sigma)."""
    lo, hi = rho_hat / ratio, rho_hat
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    rho_prev = 1.0 / sigma
    d = (dinv * r) / theta
    x = np.zeros_like(r)
    rk = r.copy()
    for _ in range(1, m):
        x = x + d
        rk = rk - A(d)
        rho = 1.0 / (2.0 * sigma - rho_prev)
        d = rho * rho_prev * d + (2.0 * rho / delta) * (dinv * rk)
        rho_prev = rho
    return x + d


def lanczos_lmax(A, dinv, v0, steps=20, project=None):
    """Largest eigenvalue of S A estimated from `steps` Jacobi-PCG iterations
    on A x = v0 through the CG-Lanczos relation: the tridiagonal T has
    T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1} = sqrt(beta_j)/alpha_j."""
    b = v0 if project is None else project(v0)
    res = pcg(A, b, _as_operator(dinv), rtol=0.0, max_iter=steps, fixed_iters=True,
              project=project)
    return lmax_from_cg_coefficients(res["alpha"], res["beta"])


def lmax_from_cg_coefficients(alpha, beta):
    m = alpha.size
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(beta[j]) / alpha[j]
    return float(np.linalg.eigvalsh(T)[-1])

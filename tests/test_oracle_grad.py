"""Pins of the oracle's adjoint gradient (O13) by central finite differences.

The loss is L = sum over free unique nodes of (x - x_target)^2 with
A(k) x = b; the adjoint gradient must agree with central differences of
solves (the loss is smooth in k and linear in b).
"""

import numpy as np
import pytest

import oracle
from sem_inputs import box_mesh, manufactured_sine, random_local_normal


def _setup(N=3, shape=(2, 2, 2), h2=1.0):
    m = box_mesh(N, shape, jitter=0.05)
    k = np.exp(0.5 * 0.6 * random_local_normal((m.E, m.P), 21))
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, N, k=k, h2=h2)
    f = manufactured_sine(m.xyz)
    b = P.rhs_from_source(f)
    target = P.num.from_local_consistent(f) / (3 * np.pi ** 2 + h2)
    return m, P, k, b, target


def _loss(P, k, b, target):
    P.set_k(k)
    x = P.solve(b, rtol=1e-14, max_iter=20000)["x"]
    return float((x - target) @ (x - target))


def test_adjoint_gradient_in_k_matches_central_differences():
    m, P, k, b, target = _setup()
    g = oracle.solve_and_adjoint_gradient(P, b, target, rtol=1e-14)
    kbar = g["kbar_local"]
    rng = np.random.default_rng(5)
    eps = 1e-4
    for _ in range(5):
        dk = k * rng.standard_normal(k.shape)
        fd = (_loss(P, k + eps * dk, b, target) - _loss(P, k - eps * dk, b, target)) / (2 * eps)
        P.set_k(k)
        ad = float(np.sum(kbar * dk))
        assert abs(fd - ad) <= 1e-6 * abs(fd), (fd, ad)


def test_adjoint_gradient_in_b_matches_central_differences():
    m, P, k, b, target = _setup()
    g = oracle.solve_and_adjoint_gradient(P, b, target, rtol=1e-14)
    rng = np.random.default_rng(6)
    eps = 1e-3
    for _ in range(3):
        db = rng.standard_normal(b.shape)
        fd = (_loss(P, k, b + eps * db, target) - _loss(P, k, b - eps * db, target)) / (2 * eps)
        assert abs(fd - g["lam"] @ db) <= 1e-7 * abs(fd)


def test_planted_sign_error_in_kbar_is_caught():
    m, P, k, b, target = _setup()
    g = oracle.solve_and_adjoint_gradient(P, b, target, rtol=1e-14)
    dk = k * np.random.default_rng(8).standard_normal(k.shape)
    eps = 1e-4
    fd = (_loss(P, k + eps * dk, b, target) - _loss(P, k - eps * dk, b, target)) / (2 * eps)
    wrong = -float(np.sum(g["kbar_local"] * dk))
    assert abs(fd - wrong) > 1e-3 * abs(fd)

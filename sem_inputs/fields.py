"""Seeded scalar fields sampled at mesh nodes (inputs only)."""

from __future__ import annotations

import numpy as np

from .meshes import BoxMesh


def manufactured_sine(xyz: np.ndarray) -> np.ndarray:
    """u(x, y, z) = sin(pi x) sin(pi y) sin(pi z) at every local node, (E, P)."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def unique_dirichlet_flags(mesh: BoxMesh) -> np.ndarray:
    """Per-unique-node Dirichlet flag (bool, length n_unique)."""
    f = np.zeros(mesh.n_unique, dtype=bool)
    if mesh.dirichlet is not None:
        f[mesh.gid[mesh.dirichlet.astype(bool)]] = True
    return f


def random_unique_normal(mesh: BoxMesh, seed: int = 2, zero_mean: bool = False) -> np.ndarray:
    """i.i.d. N(0,1) value per unique node, zero on Dirichlet nodes, optionally
    shifted to zero mean over the unique nodes; returned copy-consistent at
    every local node, (E, P)."""
    rng = np.random.default_rng(seed)
    bu = rng.standard_normal(mesh.n_unique)
    bu[unique_dirichlet_flags(mesh)] = 0.0
    if zero_mean:
        bu -= bu.mean()
    return bu[mesh.gid]


def random_fourier_field(xyz: np.ndarray, M: int = 64, ell: float = 0.2, seed: int = 3) -> np.ndarray:
    """Smooth unit-variance random field by random Fourier features:
    g(x) = sqrt(2/M) sum_m cos(2 pi kappa_m . x + phi_m),
    kappa_m ~ N(0, (1/(2 pi ell))^2 I), phi_m ~ U[0, 2 pi).
    Evaluated at the node coordinates, so it is continuous across elements."""
    rng = np.random.default_rng(seed)
    kappa = rng.normal(0.0, 1.0 / (2.0 * np.pi * ell), size=(M, 3))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=M)
    shp = xyz.shape[:-1]
    X = xyz.reshape(-1, 3)
    g = np.zeros(X.shape[0])
    for m in range(M):
        g += np.cos(2.0 * np.pi * (X @ kappa[m]) + phi[m])
    g *= np.sqrt(2.0 / M)
    return g.reshape(shp)


def velocity_field(xyz: np.ndarray, seed: int = 11, ell: float = 0.25, M: int = 32) -> np.ndarray:
    """(3, E, P): a smooth seeded velocity, one random Fourier field (seeds
    seed, seed + 1, seed + 2) per component, continuous across elements."""
    return np.stack([random_fourier_field(xyz, M=M, ell=ell, seed=seed + c) for c in range(3)])


def random_local_normal(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) per local point (not copy-consistent)."""
    return np.random.default_rng(seed).standard_normal(shape)

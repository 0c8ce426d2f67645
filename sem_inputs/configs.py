"""The five benchmark workloads as seeded recipes.

1  Poisson on the unit cube, 4x4x4 elements, N=7, interior-vertex jitter of
   +-5 % of the element size (seed 1), homogeneous Dirichlet walls, right-hand
   side from the manufactured solution sin(pi x) sin(pi y) sin(pi z).
2  One GPU's share of a convection box: [0,4]x[0,4]x[0,1], 32x32x16 elements,
   N=7, periodic in x and y, Dirichlet plates at z=0,1, tanh clustering of the
   element layers to both plates (largest/smallest height 20), smooth seeded
   deformation (a=0.15, seed 1), random normal right-hand side (seed 2).
3  Config 1 at N=7 and N=9 (precision variants of the solve).
4  Variable-coefficient Helmholtz on the unit cube, 16^3 elements, N=7,
   jitter as config 1, Dirichlet walls, k = exp(0.5 g) with g a smooth random
   field (seed 3), h2 = 1.
5  Unit cube, 32^3 elements, N=9, tanh clustering in z (ratio 20), wall-
   preserving deformation, all-Neumann boundary (constant null space), random
   normal zero-mean right-hand side (seed 2).

``shape`` may be overridden to build a smaller instance of the same recipe.
"""

from __future__ import annotations

import numpy as np

from .meshes import box_mesh, BoxMesh
from .fields import manufactured_sine, random_unique_normal, random_fourier_field

CONFIGS = {
    1: dict(N=7, shape=(4, 4, 4), lengths=(1.0, 1.0, 1.0), periodic=(False, False, False),
            dirichlet="all", jitter=0.05, z_ratio=None, deform=None, h2=0.0, rhs="sine", k=None),
    2: dict(N=7, shape=(32, 32, 16), lengths=(4.0, 4.0, 1.0), periodic=(True, True, False),
            dirichlet="z", jitter=0.0, z_ratio=20.0, deform=dict(a=0.15, seed=1, kind="periodic"),
            h2=0.0, rhs="normal", k=None),
    3: dict(N=9, shape=(4, 4, 4), lengths=(1.0, 1.0, 1.0), periodic=(False, False, False),
            dirichlet="all", jitter=0.05, z_ratio=None, deform=None, h2=0.0, rhs="sine", k=None),
    4: dict(N=7, shape=(16, 16, 16), lengths=(1.0, 1.0, 1.0), periodic=(False, False, False),
            dirichlet="all", jitter=0.05, z_ratio=None, deform=None, h2=1.0, rhs="sine", k="rff"),
    5: dict(N=9, shape=(32, 32, 32), lengths=(1.0, 1.0, 1.0), periodic=(False, False, False),
            dirichlet="none", jitter=0.0, z_ratio=20.0, deform=dict(a=0.15, seed=1, kind="walls"),
            h2=0.0, rhs="normal0", k=None),
}


def config_mesh(cfg: int, N: int | None = None, shape: tuple | None = None,
                ref_nodes: np.ndarray | None = None) -> tuple[BoxMesh, dict]:
    """Return (mesh, fields) for a workload.

    fields: 'f' pointwise source at local nodes (sine configs) or None;
    'b' copy-consistent assembled right-hand side values (random configs) or
    None; 'k' conductivity per local point or None; 'h2'.
    """
    c = dict(CONFIGS[cfg])
    if N is not None:
        c["N"] = N
    if shape is not None:
        c["shape"] = tuple(shape)
    mesh = box_mesh(c["N"], c["shape"], c["lengths"], c["periodic"], c["dirichlet"],
                    jitter=c["jitter"], jitter_seed=1, z_ratio=c["z_ratio"],
                    deform=c["deform"], ref_nodes=ref_nodes)
    f = b = k = None
    if c["rhs"] == "sine":
        f = manufactured_sine(mesh.xyz)
    elif c["rhs"] == "normal":
        b = random_unique_normal(mesh, seed=2)
    elif c["rhs"] == "normal0":
        b = random_unique_normal(mesh, seed=2, zero_mean=True)
    if c["k"] == "rff":
        k = np.exp(0.5 * random_fourier_field(mesh.xyz, seed=3))
    return mesh, dict(f=f, b=b, k=k, h2=c["h2"])

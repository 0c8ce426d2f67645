"""Seeded synthetic inputs for the spectral-element solve.

This package produces *inputs only*: hexahedral box meshes (node coordinates at
every local point, global node ids, Dirichlet flags) and scalar fields sampled
at the nodes.  It contains none of the method's arithmetic (no quadrature
weights, no derivative matrix, no geometric factors, no assembly).  Both the
CPU oracle and the HIP library consume what it produces, and neither depends
on the other.

Layout conventions shared by every consumer (the paper's tensor-product
``ijk`` ordering of the unknowns on the reference element, Sec. 2.2):

* local point index ``q = i + (N+1)*(j + (N+1)*k)``, ``i`` fastest, with
  ``i``, ``j``, ``k`` running along the reference coordinates ``r``, ``s``, ``t``;
* element index ``e = ex + nex*(ey + ney*ez)``;
* arrays of local values are ``[E][(N+1)^3]`` (C order).
"""

from .meshes import BoxMesh, box_mesh, reference_node_placement, tanh_vertices
from .fields import (
    manufactured_sine,
    random_unique_normal,
    random_fourier_field,
    random_local_normal,
    unique_dirichlet_flags,
    velocity_field,
)
from .configs import config_mesh, CONFIGS

__all__ = [
    "velocity_field",
    "BoxMesh",
    "box_mesh",
    "reference_node_placement",
    "tanh_vertices",
    "manufactured_sine",
    "random_unique_normal",
    "random_fourier_field",
    "random_local_normal",
    "unique_dirichlet_flags",
    "config_mesh",
    "CONFIGS",
]

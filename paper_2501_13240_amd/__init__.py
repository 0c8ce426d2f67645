"""MI355X-native matrix-free spectral-element Poisson/Helmholtz solve.

The hot path of the paper's convection solver (Sec. 2.2): the tensor-product
element operator on hexahedra at GLL order N, direct-stiffness summation by
sorted segmented sums, inside Jacobi- and fourth-kind-Chebyshev-preconditioned
conjugate gradients, with FP32 preconditioning / iterative refinement and a
differentiable solve.  All computation runs in ``libsem.so`` (HIP, gfx950);
this package only marshals arguments.
"""

from ._lib import LIB_PATH, load as load_library
from .api import (
    Mesh,
    SemError,
    advect,
    advection_rule,
    ax,
    ax_backward,
    cheb_apply,
    cheb_apply_noalloc,
    gll,
    gs,
    host_coarse_mesh,
    host_numbering,
    host_schwarz,
    jacobi_inverse,
    lmax_estimate,
    mask,
    mass,
    pmg_apply,
    solve,
    solve_backward,
)
from .autograd import SemSolve, sem_solve

# fail at import time, loudly, when the HIP library has not been built
load_library()

__all__ = [
    "LIB_PATH",
    "load_library",
    "Mesh",
    "SemError",
    "advect",
    "advection_rule",
    "ax",
    "ax_backward",
    "cheb_apply",
    "cheb_apply_noalloc",
    "gll",
    "gs",
    "host_coarse_mesh",
    "host_numbering",
    "host_schwarz",
    "jacobi_inverse",
    "lmax_estimate",
    "mask",
    "mass",
    "pmg_apply",
    "solve",
    "solve_backward",
    "SemSolve",
    "sem_solve",
]

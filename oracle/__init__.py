"""CPU oracle for the spectral-element Poisson/Helmholtz solve (FP64, NumPy/SciPy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP path: it consumes the
seeded inputs (coordinates, global ids, Dirichlet flags, fields) and computes
everything else itself, in plain array code that follows the method's
definitions in order:

* ``gll``       Gauss-Lobatto-Legendre nodes, weights and the derivative matrix
                (the nodal basis and quadrature of the method, Sec. 2.2);
* ``geometry``  per-point metric of the element map by the chain rule
                (Sec. 2.2), six symmetric factors G_ab and the mass B;
* ``operator``  the matrix-free tensor-product element operator
                A_e u = D^T (k G) D u + h2 B u (Sec. 2.2), its diagonal, and the
                backward (derivative in k) contraction;
* ``assembly``  direct-stiffness summation (gather-scatter, Sec. 2.2 paragraph
                on the surface exchange), restriction to free nodes, and the
                explicitly assembled sparse matrix for small meshes;
* ``solvers``   Jacobi-preconditioned conjugate gradients (the pressure Poisson
                solve, Sec. 2.2), fourth-kind Chebyshev acceleration
                (Sec. 2.2), CG-Lanczos eigenvalue bound, null-space projection;
* ``grad``      the adjoint gradient of a solve with respect to k and b;
* ``pmg``       the p-multigrid preconditioner with Chebyshev smoothing (the
                default pressure preconditioner named in Sec. 2.2);
* ``schwarz``   the overlapping Schwarz smoother with fast-diagonalisation
                local solves that the p-multigrid cycle can accelerate;
* ``advection`` the convective term u . grad T of the Boussinesq equations
                (Sec. 4.1), by GLL collocation or by the 3/2 Gauss rule.

The paper names the method but prints none of its formulas; every function
states the textbook definition it follows and each is pinned by a test under
``tests/`` against closed forms, library routines or invariants.
"""

from .gll import gll_nodes_weights, deriv_matrix, deriv_matrix_barycentric, legendre
from .geometry import geometric_factors
from .operator import (local_apply, local_diagonal, mass_apply, kgrad_contraction,
                       local_apply_lowprec, local_apply_majorant, round_to_format, block_scale)
from .assembly import Numbering, explicit_matrix, element_matrices
from .solvers import Problem, pcg, chebyshev_apply, chebyshev1_apply, lanczos_lmax
from .pmg import PMG, coarse_mesh, interpolation_matrix, level_orders
from .schwarz import Schwarz, extended_1d
from .grad import solve_and_adjoint_gradient
from .advection import convect, dealias_points, geometric_factors_q, lagrange_at

__all__ = [
    "convect",
    "dealias_points",
    "geometric_factors_q",
    "lagrange_at",
    "gll_nodes_weights",
    "deriv_matrix",
    "deriv_matrix_barycentric",
    "legendre",
    "geometric_factors",
    "local_apply",
    "local_diagonal",
    "mass_apply",
    "kgrad_contraction",
    "local_apply_lowprec",
    "local_apply_majorant",
    "round_to_format",
    "block_scale",
    "Numbering",
    "explicit_matrix",
    "element_matrices",
    "Problem",
    "pcg",
    "chebyshev_apply",
    "chebyshev1_apply",
    "lanczos_lmax",
    "solve_and_adjoint_gradient",
    "PMG",
    "coarse_mesh",
    "interpolation_matrix",
    "level_orders",
    "Schwarz",
    "extended_1d",
]

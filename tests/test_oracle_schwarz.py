"""Pins of the oracle's overlapping Schwarz smoother (the smoother family
Sec. 2.2 names for p-multigrid; readings in oracle/schwarz.py).

Pins: the subdomain map equals the structured lattice of the box generator
(face-extension points = the neighbour's node one step inside, edge and
corner points absent); on brick meshes, where the assembled operator
restricted to an extended box is exactly separable (also with clustered
layers of different heights), the fast-diagonalisation solve equals a dense
solve of that principal submatrix, for interior and boundary elements, with
Neumann and Dirichlet walls; the additive operator is symmetric positive
definite; Chebyshev-accelerated Schwarz smoothing gives p-multigrid fewer
iterations than Jacobi smoothing on a clustered deformed box.
"""

import numpy as np
import pytest

import oracle
from oracle.assembly import explicit_matrix
from oracle.pmg import PMG
from oracle.schwarz import Schwarz
from oracle.solvers import Problem
from sem_inputs import box_mesh, config_mesh


def _lattice_gid(shape, N, periodic, e, pt):
    """Structured global id of lattice point pt = (i, j, k) of element e, or
    None outside a non-periodic lattice (the box generator's numbering)."""
    nex, ney, nez = shape
    ec = (e % nex, (e // nex) % ney, e // (nex * ney))
    g, size = [], []
    for d in range(3):
        v = ec[d] * N + pt[d]
        n = shape[d] * N
        if periodic[d]:
            v %= n
            size.append(n)
        else:
            if v < 0 or v > n:
                return None
            size.append(n + 1)
        g.append(v)
    return g[0] + size[0] * (g[1] + size[1] * g[2])


@pytest.mark.parametrize("periodic,dirichlet", [((True, False, False), "none"),
                                                ((False, False, False), "all"),
                                                ((True, True, False), "z")])
def test_subdomain_map_equals_the_structured_lattice(periodic, dirichlet):
    N, shape = 3, (3, 3, 3)
    m = box_mesh(N, shape, (1.0, 1.3, 0.8), periodic=periodic, dirichlet=dirichlet, jitter=0.05)
    P = Problem(m.xyz, m.gid, m.dirichlet, N)
    S = Schwarz(m.xyz, m.gid, m.dirichlet, N, P.num)
    gid_of_free = P.num.gids[P.num.free]
    nx = N + 3
    ext = S.ext.reshape(m.E, nx, nx, nx)
    dir_u = set(P.num.gids[P.num.dirichlet_u].tolist())
    for e in range(m.E):
        for k in range(-1, N + 2):
            for j in range(-1, N + 2):
                for i in range(-1, N + 2):
                    out = sum(c < 0 or c > N for c in (i, j, k))
                    got = ext[e, k + 1, j + 1, i + 1]
                    if out >= 2:
                        assert got == -1
                        continue
                    want = _lattice_gid(shape, N, periodic, e, (i, j, k))
                    if want is None or want in dir_u:
                        assert got == -1, (e, i, j, k)
                    else:
                        assert got >= 0 and gid_of_free[got] == want, (e, i, j, k)


@pytest.mark.parametrize("dirichlet", ["none", "all"])
def test_fast_diagonalisation_is_exact_on_brick_boxes(dirichlet):
    N, shape = 3, (4, 3, 4)
    periodic = (False, False, False)
    m = box_mesh(N, shape, (1.0, 1.6, 0.8), periodic=periodic, dirichlet=dirichlet, z_ratio=3.0)
    P = Problem(m.xyz, m.gid, m.dirichlet, N)
    S = Schwarz(m.xyz, m.gid, m.dirichlet, N, P.num)
    A = explicit_matrix(P.G, P.B, N, P.num).toarray()  # free nodes
    free_pos = {int(g): f for f, g in enumerate(P.num.gids[P.num.free])}
    nx = N + 3
    rng = np.random.default_rng(3)
    for e in (0, 5, 13, 22, m.E - 1):  # corner, edge, interior and face elements
        pts, rows = [], []
        for k in range(-1, N + 2):
            for j in range(-1, N + 2):
                for i in range(-1, N + 2):
                    g = _lattice_gid(shape, N, periodic, e, (i, j, k))
                    if g is not None and g in free_pos:
                        pts.append((k + 1) * nx * nx + (j + 1) * nx + (i + 1))
                        rows.append(free_pos[g])
        pts, rows = np.array(pts), np.array(rows)
        rbox = np.zeros((m.E, nx ** 3))
        rbox[e, pts] = rng.standard_normal(pts.size)
        z = S.local_solve(rbox)[e, pts]
        ref = np.linalg.solve(A[np.ix_(rows, rows)], rbox[e, pts])
        assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref), e


def test_schwarz_is_symmetric_positive_definite():
    m = box_mesh(4, (3, 3, 4), (1.0, 1.0, 1.0), periodic=(True, False, False), dirichlet="z",
                 jitter=0.05, z_ratio=4.0, deform=dict(a=0.15, seed=2, kind="walls"))
    P = Problem(m.xyz, m.gid, m.dirichlet, 4)
    S = Schwarz(m.xyz, m.gid, m.dirichlet, 4, P.num)
    rng = np.random.default_rng(4)
    for _ in range(3):
        x, y = rng.standard_normal(P.num.n_free), rng.standard_normal(P.num.n_free)
        Sx, Sy = S.apply(x), S.apply(y)
        assert abs(Sx @ y - x @ Sy) <= 1e-12 * np.linalg.norm(Sx) * np.linalg.norm(y)
        assert Sx @ x > 0


def test_schwarz_smoothing_beats_jacobi_smoothing_on_a_clustered_box():
    m, fld = config_mesh(5, shape=(6, 6, 6))
    jac = PMG(m.xyz, m.gid, m.dirichlet, m.N, smoother="jacobi")
    sch = PMG(m.xyz, m.gid, m.dirichlet, m.N, smoother="schwarz")
    b = jac.levels[0].num.from_local_consistent(fld["b"])
    b -= b.mean()
    rj, rs = jac.solve(b, rtol=1e-10), sch.solve(b, rtol=1e-10)
    assert rj["converged"] and rs["converged"]
    assert rs["iters"] < rj["iters"], (rs["iters"], rj["iters"])
    assert np.linalg.norm(rs["x"] - rj["x"]) <= 1e-8 * np.linalg.norm(rj["x"])

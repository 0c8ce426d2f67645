"""Seeded hexahedral box meshes.

A mesh is described by what a spectral-element code receives: the physical
coordinates of every local node of every element, a global id per local node
(equal ids = the same global unknown; periodicity is expressed this way) and a
per-local-node Dirichlet flag.

Node placement inside an element: the trilinear image of the tensor-product
Gauss-Lobatto-Legendre points of the reference cube [-1,1]^3 (the nodal set of
the method, Sec. 2.2), optionally followed by a smooth deformation applied to
all nodes.  The reference points are obtained here from numpy's Legendre
root finder (interior points = roots of P_N'), which is part of the *input
recipe*: the solver under test computes its own quadrature from the order N.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import legendre as _leg


def reference_node_placement(N: int) -> np.ndarray:
    """1-D node placement on [-1, 1]: endpoints plus the roots of P_N'.

    Made exactly antisymmetric so that meshes are mirror-symmetric.
    """
    if N < 1:
        raise ValueError("N must be >= 1")
    if N == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(N + 1)
    c[N] = 1.0
    r = np.sort(np.real(_leg.legroots(_leg.legder(c))))
    r = 0.5 * (r - r[::-1])
    return np.concatenate([[-1.0], r, [1.0]])


def tanh_vertices(n: int, ratio: float) -> tuple[np.ndarray, float]:
    """Element-vertex coordinates on [0, 1] clustered towards both ends.

    z_m = (1 + tanh(g (2m/n - 1)) / tanh(g)) / 2, m = 0..n, with the
    stretching parameter g found by bisection so that the largest element
    height is ``ratio`` times the smallest.  Returns (vertices, g).
    """
    if ratio <= 1.0:
        return np.linspace(0.0, 1.0, n + 1), 0.0
    m = np.arange(n + 1)

    def verts(g):
        return 0.5 * (1.0 + np.tanh(g * (2.0 * m / n - 1.0)) / np.tanh(g))

    def r_of(g):
        d = np.diff(verts(g))
        return d.max() / d.min()

    lo, hi = 1e-3, 10.0
    if r_of(hi) < ratio:
        raise ValueError(f"ratio {ratio} not reachable with {n} elements")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if r_of(mid) < ratio:
            lo = mid
        else:
            hi = mid
    g = 0.5 * (lo + hi)
    v = verts(g)
    v[0], v[-1] = 0.0, 1.0
    return v, g


@dataclass
class BoxMesh:
    """A box mesh of ``nex*ney*nez`` hexahedra at order N (see module doc)."""

    N: int
    shape: tuple
    lengths: tuple
    periodic: tuple
    xyz: np.ndarray  # (E, (N+1)^3, 3) float64
    gid: np.ndarray  # (E, (N+1)^3) int64
    dirichlet: np.ndarray | None  # (E, (N+1)^3) uint8, or None
    n_unique: int
    meta: dict = field(default_factory=dict)

    @property
    def E(self) -> int:
        return self.xyz.shape[0]

    @property
    def P(self) -> int:
        return (self.N + 1) ** 3


def _vertex_lattice(shape, lengths, z_ratio):
    nex, ney, nez = shape
    vx = np.linspace(0.0, lengths[0], nex + 1)
    vy = np.linspace(0.0, lengths[1], ney + 1)
    gamma = 0.0
    if z_ratio is not None and z_ratio > 1.0:
        vz, gamma = tanh_vertices(nez, z_ratio)
        vz = vz * lengths[2]
    else:
        vz = np.linspace(0.0, lengths[2], nez + 1)
    V = np.empty((nex + 1, ney + 1, nez + 1, 3))
    V[..., 0] = vx[:, None, None]
    V[..., 1] = vy[None, :, None]
    V[..., 2] = vz[None, None, :]
    return V, (vx, vy, vz), gamma


def _jitter(V, spacing, amount, seed):
    """Uniform i.i.d. displacement in [-amount*h, amount*h] per coordinate of
    every vertex strictly inside the box; h is the smaller adjacent spacing."""
    rng = np.random.default_rng(seed)
    out = V.copy()
    hs = []
    for d, v in enumerate(spacing):
        dv = np.diff(v)
        h = np.minimum(np.concatenate([[np.inf], dv]), np.concatenate([dv, [np.inf]]))
        hs.append(h)
    nx, ny, nz = V.shape[:3]
    disp = rng.uniform(-1.0, 1.0, size=V.shape)
    interior = np.zeros((nx, ny, nz), dtype=bool)
    interior[1:-1, 1:-1, 1:-1] = True
    for d in range(3):
        hd = hs[d]
        shp = [1, 1, 1]
        shp[d] = -1
        out[..., d] += np.where(interior, amount * disp[..., d] * hd.reshape(shp), 0.0)
    return out


def box_mesh(
    N: int,
    shape: tuple,
    lengths: tuple = (1.0, 1.0, 1.0),
    periodic: tuple = (False, False, False),
    dirichlet: str = "all",
    jitter: float = 0.0,
    jitter_seed: int = 1,
    z_ratio: float | None = None,
    deform: dict | None = None,
    ref_nodes: np.ndarray | None = None,
    chunk: int = 4096,
) -> BoxMesh:
    """Build a seeded box mesh.

    dirichlet: 'all' (every non-periodic wall), 'z' (bottom and top plates
    only) or 'none' (pure Neumann; returns ``dirichlet=None``).
    deform: None or dict(a=..., seed=..., kind='periodic'|'walls'), the smooth
    horizontal displacement that vanishes at the plates z = 0, Lz:
      periodic: x += a*hx*sin(2 pi y/Ly + p1)*sin(pi z/Lz),
                y += a*hy*sin(2 pi x/Lx + p2)*sin(pi z/Lz)
      walls:    the same times sin(pi x/Lx) (for x) and sin(pi y/Ly) (for y),
                so the side walls stay planar.
    """
    nex, ney, nez = shape
    E = nex * ney * nez
    n1 = N + 1
    xi = reference_node_placement(N) if ref_nodes is None else np.asarray(ref_nodes, float)
    assert xi.shape == (n1,)

    V, spacing, gamma = _vertex_lattice(shape, lengths, z_ratio)
    if jitter > 0.0:
        V = _jitter(V, spacing, jitter, jitter_seed)

    # trilinear shape functions at the reference nodes: lo/hi corner weights
    l1 = np.stack([(1.0 - xi) / 2.0, (1.0 + xi) / 2.0])  # (2, N+1)

    ex = np.arange(E) % nex
    ey = (np.arange(E) // nex) % ney
    ez = np.arange(E) // (nex * ney)

    xyz = np.empty((E, n1, n1, n1, 3))
    for s in range(0, E, chunk):
        sl = slice(s, min(E, s + chunk))
        cx, cy, cz = ex[sl], ey[sl], ez[sl]
        # corners C[e, cz, cy, cx, d]
        C = np.empty((cx.size, 2, 2, 2, 3))
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    C[:, a, b, c, :] = V[cx + c, cy + b, cz + a, :]
        xyz[sl] = np.einsum("zk,yj,xi,ezyxd->ekjid", l1, l1, l1, C, optimize=True)

    if deform is not None:
        a = float(deform["a"])
        rng = np.random.default_rng(int(deform.get("seed", 1)))
        p1, p2 = rng.uniform(0.0, 2.0 * np.pi, size=2)
        hx, hy = lengths[0] / nex, lengths[1] / ney
        Lx, Ly, Lz = lengths
        X, Y, Z = xyz[..., 0].copy(), xyz[..., 1].copy(), xyz[..., 2].copy()
        sz = np.sin(np.pi * Z / Lz)
        dx = a * hx * np.sin(2.0 * np.pi * Y / Ly + p1) * sz
        dy = a * hy * np.sin(2.0 * np.pi * X / Lx + p2) * sz
        if deform.get("kind", "periodic") == "walls":
            dx = dx * np.sin(np.pi * X / Lx)
            dy = dy * np.sin(np.pi * Y / Ly)
        xyz[..., 0] = X + dx
        xyz[..., 1] = Y + dy
        deform = dict(deform, phases=(float(p1), float(p2)))

    xyz = xyz.reshape(E, n1 ** 3, 3)

    # global node lattice indices
    i = np.arange(n1)
    gx = (ex[:, None, None, None] * N + i[None, None, None, :])
    gy = (ey[:, None, None, None] * N + i[None, None, :, None])
    gz = (ez[:, None, None, None] * N + i[None, :, None, None])
    gx = np.broadcast_to(gx, (E, n1, n1, n1)).astype(np.int64)
    gy = np.broadcast_to(gy, (E, n1, n1, n1)).astype(np.int64)
    gz = np.broadcast_to(gz, (E, n1, n1, n1)).astype(np.int64)
    G = []
    for d, (g, ne) in enumerate(zip((gx, gy, gz), shape)):
        if periodic[d]:
            g = g % (ne * N)
            G.append((g, ne * N))
        else:
            G.append((g, ne * N + 1))
    (gx, GX), (gy, GY), (gz, GZ) = G
    gid = (gx + GX * (gy + GY * gz)).reshape(E, n1 ** 3)
    n_unique = GX * GY * GZ

    if dirichlet == "none":
        dmask = None
    else:
        walls = np.zeros((E, n1, n1, n1), dtype=bool)
        dirs = (0, 1, 2) if dirichlet == "all" else (2,) if dirichlet == "z" else None
        if dirs is None:
            raise ValueError(f"unknown dirichlet kind {dirichlet!r}")
        for d in dirs:
            g, Gd = G[d]
            if periodic[d]:
                continue
            walls |= (g == 0) | (g == Gd - 1)
        dmask = walls.reshape(E, n1 ** 3).astype(np.uint8)

    meta = dict(gamma=gamma, jitter=jitter, jitter_seed=jitter_seed,
                z_ratio=z_ratio, deform=deform)
    return BoxMesh(N=N, shape=tuple(shape), lengths=tuple(lengths),
                   periodic=tuple(periodic), xyz=xyz, gid=gid,
                   dirichlet=dmask, n_unique=int(n_unique), meta=meta)

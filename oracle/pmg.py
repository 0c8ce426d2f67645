"""p-multigrid preconditioner for the pressure-type solve.

Test infrastructure only (see the package docstring).

Sec. 2.2 names the default preconditioner of the pressure Poisson solve:
p-multigrid whose smoothing is accelerated by fourth-kind Chebyshev
polynomials, with most preconditioner work in FP32.  It prints no further
detail; the readings taken here are:

* levels of polynomial order N_0 = N, N_{l+1} = floor(N_l / 2), ..., 1 on the
  same hexahedra;
* the coarse element maps interpolate the fine ones at the coarse GLL points,
  and each level's operator is the same spectral-element operator assembled
  from that geometry (the coarse problem is rediscretised);
* coarse unknowns are identified across elements through the fine mesh's
  global ids (periodicity carries over through equal ids): a coarse node is a
  mesh vertex, a position along a mesh edge, a position on a mesh face, or an
  element-interior position;
* prolongation P_l interpolates a coarse element block to the fine GLL points
  (tensor product of the 1-D Lagrange interpolation J_l); restriction is its
  transpose in the unique-node inner product;
* smoothing (pre and post) is the fourth-kind Chebyshev-Jacobi polynomial of
  order m with bound rho_hat_l = 1.1 x a 20-step CG-Lanczos estimate of
  lambda_max(S_l A_l); the coarsest level runs a fixed number of Jacobi-PCG
  iterations from zero (with the constant mode projected out when it is
  singular);
* the V-cycle
      V_l(r): x = Cheb_l(r); x += P_l V_{l+1}(P_l^T (r - A_l x));
              x += Cheb_l(r - A_l x)
  preconditions a flexible CG.
"""

from __future__ import annotations

import numpy as np

from .gll import gll_nodes_weights
from .geometry import tensor
from .solvers import Problem, chebyshev_apply, lanczos_lmax, pcg


def level_orders(N: int) -> list[int]:
    """N, floor(N/2), ..., 1."""
    out = [N]
    while out[-1] > 1:
        out.append(out[-1] // 2)
    return out


def interpolation_matrix(n_from: int, n_to: int) -> np.ndarray:
    """(n_to+1) x (n_from+1) matrix of the Lagrange basis on the GLL nodes of
    order n_from evaluated at the GLL nodes of order n_to (barycentric form)."""
    xf, _ = gll_nodes_weights(n_from)
    xt, _ = gll_nodes_weights(n_to)
    diff = xf[:, None] - xf[None, :]
    np.fill_diagonal(diff, 1.0)
    lam = 1.0 / np.prod(diff, axis=1)  # barycentric weights
    J = np.zeros((xt.size, xf.size))
    for i, x in enumerate(xt):
        d = x - xf
        hit = np.flatnonzero(d == 0.0)
        if hit.size:
            J[i, hit[0]] = 1.0
            continue
        t = lam / d
        J[i] = t / t.sum()
    return J


def tensor_apply(M: np.ndarray, X: np.ndarray) -> np.ndarray:
    """(M x M x M) applied to every element block: X (E, (n+1)^3) in ijk order
    -> (E, (m+1)^3) with M of shape (m+1, n+1)."""
    n = M.shape[1] - 1
    T = tensor(X, n)  # (E, k, j, i)
    T = np.einsum("ai,ekji->ekja", M, T)
    T = np.einsum("bj,ekja->ekba", M, T)
    T = np.einsum("ck,ekba->ecba", M, T)
    return T.reshape(X.shape[0], -1)


def coarse_mesh(xyz: np.ndarray, gid: np.ndarray, dirichlet, N: int, Nc: int):
    """Coordinates, global ids and Dirichlet flags of the order-Nc mesh on the
    same hexahedra (see the module docstring).  Python loops: small meshes."""
    E = xyz.shape[0]
    I = interpolation_matrix(N, Nc)
    xyz_c = np.stack([tensor_apply(I, np.ascontiguousarray(xyz[:, :, c])) for c in range(3)], -1)
    n, nc = N + 1, Nc + 1
    g = gid.reshape(E, n, n, n)  # [e, k, j, i]
    dfl = None if dirichlet is None else dirichlet.reshape(E, n, n, n)

    def fine_pos(c):
        # coarse index 0 / Nc -> fine 0 / N; interior coarse positions keep a
        # fine interior position (index 1) for the entity's Dirichlet flag
        return 0 if c == 0 else N if c == Nc else 1

    keys = {}
    gid_c = np.empty((E, nc, nc, nc), dtype=np.int64)
    dir_c = np.zeros((E, nc, nc, nc), dtype=np.uint8)
    for e in range(E):
        for k in range(nc):
            for j in range(nc):
                for i in range(nc):
                    c = (i, j, k)
                    on = [ci in (0, Nc) for ci in c]
                    nb = sum(on)
                    if nb == 3:
                        key = ("v", int(g[e, fine_pos(k), fine_pos(j), fine_pos(i)]))
                    elif nb == 2:
                        d = on.index(False)  # the edge runs along direction d

                        def end(t, d=d):
                            q = [fine_pos(x) for x in c]
                            q[d] = t
                            return int(g[e, q[2], q[1], q[0]])
                        g0, g1 = end(0), end(N)
                        if g0 == g1:
                            raise ValueError("an edge whose ends share a global id")
                        t = c[d]
                        key = ("e", g0, g1, t) if g0 < g1 else ("e", g1, g0, Nc - t)
                    elif nb == 1:
                        d = on.index(True)  # the face is normal to direction d
                        d1, d2 = [x for x in range(3) if x != d]

                        def corner(a, b, d1=d1, d2=d2):
                            q = [fine_pos(x) for x in c]
                            q[d1], q[d2] = (0 if a == 0 else N), (0 if b == 0 else N)
                            return int(g[e, q[2], q[1], q[0]])
                        cs = {(a, b): corner(a, b) for a in (0, 1) for b in (0, 1)}
                        if len(set(cs.values())) < 4:
                            raise ValueError("a face whose corners share a global id")
                        o = min(cs, key=cs.get)  # origin corner
                        na, nb_ = (1 - o[0], o[1]), (o[0], 1 - o[1])
                        # first axis towards the neighbour corner with the smaller id
                        if cs[na] < cs[nb_]:
                            ax1, ax2 = 0, 1
                        else:
                            ax1, ax2 = 1, 0
                        pos = (c[d1], c[d2])
                        # coordinate measured from the origin corner along each face axis
                        rel = [pos[0] if o[0] == 0 else Nc - pos[0],
                               pos[1] if o[1] == 0 else Nc - pos[1]]
                        key = ("f", cs[o], cs[na] if ax1 == 0 else cs[nb_],
                               cs[nb_] if ax1 == 0 else cs[na], rel[ax1], rel[ax2])
                    else:
                        key = ("i", e, i, j, k)
                    if key not in keys:
                        keys[key] = len(keys)
                    gid_c[e, k, j, i] = keys[key]
                    if dfl is not None and nb > 0:
                        q = [fine_pos(x) for x in c]
                        dir_c[e, k, j, i] = dfl[e, q[2], q[1], q[0]]
    P = nc ** 3
    return (xyz_c, gid_c.reshape(E, P),
            None if dirichlet is None else dir_c.reshape(E, P))


def fixed_pcg(A, b, dinv, iters, project=None):
    """`iters` Jacobi-PCG iterations from x = 0 (r projected when `project`
    is given); stops early, keeping the iterate, when p.Ap <= 0 (the residual
    has vanished)."""
    x = np.zeros_like(b)
    r = b.copy() if project is None else project(b)
    z = dinv * r
    p = z.copy()
    rho = r @ z
    if not rho > 0.0:
        return x
    for _ in range(iters):
        w = A(p)
        pw = p @ w
        if not pw > 0.0:
            break
        alpha = rho / pw
        x = x + alpha * p
        r = r - alpha * w
        if project is not None:
            r = project(r)
        z = dinv * r
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x


class PMG:
    """The level hierarchy and the V-cycle (FP64)."""

    def __init__(self, xyz, gid, dirichlet, N, k=None, h2=0.0, orders=None, smooth_order=4,
                 coarse_iters=30, coarse="cg", rho=None, smoother="schwarz"):
        self.orders = level_orders(N) if orders is None else list(orders)
        self.m = smooth_order
        self.coarse_iters = coarse_iters
        self.coarse = coarse
        self.levels = []
        for l, Nl in enumerate(self.orders):
            if l == 0:
                x_l, g_l, d_l, k_l = xyz, gid, dirichlet, k
            else:
                x_l, g_l, d_l = coarse_mesh(xyz, gid, dirichlet, N, Nl)
                k_l = None if k is None else tensor_apply(interpolation_matrix(N, Nl), k)
            self.levels.append(Problem(x_l, g_l, d_l, Nl, k=k_l, h2=h2))
        self.J = [interpolation_matrix(self.orders[l + 1], self.orders[l])
                  for l in range(len(self.orders) - 1)]
        self.dinv = [1.0 / P.diag() for P in self.levels]
        # the operator S of each smoothing level: the Jacobi diagonal, or the
        # overlapping Schwarz smoother (its coordinates and ids per level)
        self.smoother = smoother
        if smoother == "jacobi":
            self.S = list(self.dinv[:-1])
        elif smoother == "schwarz":
            from .schwarz import Schwarz
            self.S = []
            for l in range(len(self.orders) - 1):
                if l == 0:
                    x_l, g_l, d_l = xyz, gid, dirichlet
                else:
                    x_l, g_l, d_l = coarse_mesh(xyz, gid, dirichlet, N, self.orders[l])
                self.S.append(Schwarz(x_l, g_l, d_l, self.orders[l], self.levels[l].num).apply)
        else:
            raise ValueError(smoother)
        if rho is not None:  # given bounds (e.g. another implementation's estimates)
            self.rho = [float(v) for v in rho]
        else:
            self.rho = []
            for l, P in enumerate(self.levels):
                proj = P.project if P.neumann else None
                v0 = np.random.default_rng(7 + l).standard_normal(P.num.n_free)
                Sl = self.S[l] if l < len(self.S) else self.dinv[l]
                self.rho.append(1.1 * lanczos_lmax(P.apply, Sl, v0, 20, proj))
        if coarse == "exact":
            from .assembly import explicit_matrix
            Pc = self.levels[-1]
            self.Ac = explicit_matrix(Pc.G, Pc.B, Pc.N, Pc.num, k=Pc.k, h2=Pc.h2).toarray()

    def prolong(self, l, xc):
        """Level l+1 free vector -> level l free vector."""
        fine, coarse = self.levels[l], self.levels[l + 1]
        vl = tensor_apply(self.J[l], coarse.num.to_local(xc))
        return fine.num.from_local_consistent(vl)

    def restrict(self, l, rf):
        """Transpose of prolong in the unique-node inner product."""
        fine, coarse = self.levels[l], self.levels[l + 1]
        num = fine.num
        wl = num.Q(num.Rt(rf) / num.mult)
        return coarse.num.R(coarse.num.Qt(tensor_apply(self.J[l].T, wl)))

    def coarse_solve(self, r):
        P = self.levels[-1]
        if self.coarse == "exact":
            if P.neumann:
                x = np.linalg.lstsq(self.Ac, r - r.mean(), rcond=None)[0]
                return x - x.mean()
            return np.linalg.solve(self.Ac, r)
        return fixed_pcg(P.apply, r, self.dinv[-1], self.coarse_iters,
                         P.project if P.neumann else None)

    def vcycle(self, r, l=0):
        if l == len(self.levels) - 1:
            return self.coarse_solve(r)
        P = self.levels[l]
        smooth = lambda v: chebyshev_apply(P.apply, self.S[l], v, self.m, self.rho[l])
        x = smooth(r)
        x = x + self.prolong(l, self.vcycle(self.restrict(l, r - P.apply(x)), l + 1))
        return x + smooth(r - P.apply(x))

    def solve(self, b, rtol=1e-10, max_iter=1000):
        """Flexible CG on level 0 preconditioned by one V-cycle per iteration."""
        P = self.levels[0]
        proj = P.project if P.neumann else None
        if P.neumann:
            b = b - b.mean()
        res = pcg(P.apply, b, self.vcycle, rtol=rtol, max_iter=max_iter, flexible=True,
                  project=proj)
        if P.neumann:
            res["x"] = res["x"] - res["x"].mean()
        return res

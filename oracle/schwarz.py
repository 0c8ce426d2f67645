"""Overlapping Schwarz smoother with fast-diagonalisation local solves.

Test infrastructure only (see the package docstring).

Sec. 2.2 names the default pressure preconditioner: p-multigrid with
fourth-kind Chebyshev acceleration of overlapping Schwarz smoothers.  It
prints no formula; the readings taken here follow the classical minimal-
overlap spectral-element Schwarz method:

* subdomain of an element: its (N+1)^3 nodes plus, across each of its six
  faces, the layer of nodes of the neighbouring element one GLL step away
  from the shared face.  The local problem lives on the (N+3)^3 tensor box
  of these points; its edge and corner points (two or three indices outside
  0..N) take no residual and return nothing (the elements diagonally across
  an edge are not unique on general hexahedral meshes);
* local operator: the separable approximation
      A~ = B~_t x B~_s x A~_r + B~_t x A~_s x B~_r + A~_t x B~_s x B~_r
  whose 1-D factors along direction d come from three 1-D GLL elements
  [left neighbour | element | right neighbour] of the mean lengths of the
  three elements along d (stiffness (2/l) D^T diag(rho) D, mass
  (l/2) diag(rho)), assembled and restricted to the N+3 central points
  (homogeneous Dirichlet beyond them).  A side without a neighbour gets a
  decoupled ghost point (unit row); a Dirichlet face decouples the
  element's own boundary points as well;
* the inverse by fast diagonalisation: with A~_d S_d = B~_d S_d L_d and
  S_d^T B~_d S_d = I,  A~^{-1} = (S_t x S_s x S_r)
  diag(1 / (l_r,i + l_s,j + l_t,k)) (S_t x S_s x S_r)^T;
* additive combination z = sum_e R_e^T A~_e^{-1} R_e r (symmetric).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .gll import gll_nodes_weights, deriv_matrix


def _mean_lengths(xyz, N):
    """(E, 3) mean distance between opposite faces along r, s, t, from the
    corner vertices (the four element edges along each direction)."""
    E = xyz.shape[0]
    n = N + 1
    X = xyz.reshape(E, n, n, n, 3)  # [e, k, j, i, c]
    c = [0, N]
    L = np.zeros((E, 3))
    for a in c:
        for b in c:
            L[:, 0] += np.linalg.norm(X[:, a, b, N] - X[:, a, b, 0], axis=-1)
            L[:, 1] += np.linalg.norm(X[:, a, N, b] - X[:, a, 0, b], axis=-1)
            L[:, 2] += np.linalg.norm(X[:, N, a, b] - X[:, 0, a, b], axis=-1)
    return L / 4.0


def _face_index(d, side, N):
    """Local (i, j, k) tuples of the face normal to direction d at index 0
    (side 0) or N (side 1), as a function of the two tangential indices."""
    def idx(a, b):
        q = [None, None, None]
        t = [x for x in range(3) if x != d]
        q[d] = 0 if side == 0 else N
        q[t[0]], q[t[1]] = a, b
        return tuple(q)
    return idx


def extended_1d(N, l_left, l, l_right, dir_lo=False, dir_hi=False):
    """(A~, B~) of size N+3 along one direction (see the module docstring);
    l_left / l_right None: no neighbour on that side."""
    _, rho = gll_nodes_weights(N)
    D = deriv_matrix(N)
    Kh = D.T @ np.diag(rho) @ D
    Bh = np.diag(rho)
    n3 = 3 * N + 1
    A = np.zeros((n3, n3))
    B = np.zeros((n3, n3))
    for e, le in enumerate((l_left if l_left else l, l, l_right if l_right else l)):
        s = slice(e * N, e * N + N + 1)
        A[s, s] += (2.0 / le) * Kh
        B[s, s] += (le / 2.0) * Bh
    keep = np.arange(N - 1, 2 * N + 2)  # left neighbour's node N-1 .. right neighbour's node 1
    A = A[np.ix_(keep, keep)]
    B = B[np.ix_(keep, keep)]
    # an element boundary point without a neighbour keeps only its own element's
    # contribution (natural condition); the ghost beyond it is decoupled
    if l_left is None:
        A[1, 1] -= (2.0 / l) * Kh[N, N]
        B[1, 1] -= (l / 2.0) * Bh[N, N]
    if l_right is None:
        A[N + 1, N + 1] -= (2.0 / l) * Kh[0, 0]
        B[N + 1, N + 1] -= (l / 2.0) * Bh[0, 0]
    decouple = []
    if l_left is None:
        decouple.append(0)
    if l_right is None:
        decouple.append(N + 2)
    if dir_lo:
        decouple.append(1)
    if dir_hi:
        decouple.append(N + 1)
    for p in decouple:
        A[p, :] = A[:, p] = 0.0
        B[p, :] = B[:, p] = 0.0
        A[p, p] = B[p, p] = 1.0
    return A, B


class Schwarz:
    """Additive overlapping Schwarz with fast-diagonalisation local solves on
    the free unique nodes of a mesh (gid, dirichlet; free numbering `num`)."""

    def __init__(self, xyz, gid, dirichlet, N, num):
        E = gid.shape[0]
        n, nx = N + 1, N + 3
        self.N, self.E, self.nx = N, E, nx
        g = gid.reshape(E, n, n, n)
        dfl = None if dirichlet is None else dirichlet.reshape(E, n, n, n).astype(bool)
        free_of = np.full(num.n, -1, dtype=np.int64)
        free_of[num.free] = np.arange(num.n_free)
        fl = free_of[num.lid].reshape(E, n, n, n)  # free index of every local point or -1
        lengths = _mean_lengths(xyz, N)

        # faces -> (element, direction, side); a face is named by its corner ids
        faces = {}
        for e in range(E):
            for d in range(3):
                for side in (0, 1):
                    idx = _face_index(d, side, N)
                    key = frozenset(int(g[e][idx(a, b)[::-1]]) for a in (0, N) for b in (0, N))
                    if len(key) < 4:
                        raise ValueError("a face whose corners share a global id")
                    faces.setdefault(key, []).append((e, d, side))

        ext = np.full((E, nx, nx, nx), -1, dtype=np.int64)  # [e, k+1, j+1, i+1]
        ext[:, 1:-1, 1:-1, 1:-1] = fl
        self.S = np.zeros((E, 3, nx, nx))
        self.lam = np.zeros((E, 3, nx))
        for e in range(E):
            nbr_len = [[None, None], [None, None], [None, None]]
            dir_face = [[False, False], [False, False], [False, False]]
            for d in range(3):
                for side in (0, 1):
                    idx = _face_index(d, side, N)
                    key = frozenset(int(g[e][idx(a, b)[::-1]]) for a in (0, N) for b in (0, N))
                    if dfl is not None:
                        dir_face[d][side] = all(dfl[e][idx(a, b)[::-1]]
                                                for a in range(n) for b in range(n))
                    others = [f for f in faces[key] if f[0] != e or (f[1], f[2]) != (d, side)]
                    if len(others) > 1:
                        raise ValueError("a face shared by more than two elements")
                    if not others:
                        continue
                    en, dn, sn = others[0]
                    nbr_len[d][side] = lengths[en, dn]
                    # the neighbour's node one step inside, for each of our face nodes
                    nidx = _face_index(dn, sn, N)
                    where = {int(g[en][nidx(a, b)[::-1]]): nidx(a, b)
                             for a in range(n) for b in range(n)}
                    step = 1 if sn == 0 else -1
                    for a in range(n):
                        for b in range(n):
                            q = idx(a, b)  # (i, j, k) on our face
                            qn = list(where[int(g[e][q[::-1]])])
                            qn[dn] += step
                            ev = list(q)
                            ev[d] = -1 if side == 0 else N + 1
                            ext[e, ev[2] + 1, ev[1] + 1, ev[0] + 1] = fl[en][tuple(qn[::-1])]
            for d in range(3):
                A, B = extended_1d(N, nbr_len[d][0], lengths[e, d], nbr_len[d][1],
                                   dir_face[d][0], dir_face[d][1])
                lam, S = sla.eigh(A, B)
                self.S[e, d], self.lam[e, d] = S, lam
        self.ext = ext.reshape(E, -1)

    def local_solve(self, rbox):
        """A~_e^{-1} on boxes (E, (N+3)^3)."""
        E, nx = self.E, self.nx
        X = rbox.reshape(E, nx, nx, nx)  # [e, k, j, i]
        Sr, Ss, St = self.S[:, 0], self.S[:, 1], self.S[:, 2]
        X = np.einsum("eia,ekji->ekja", Sr, X)  # S_r^T along i
        X = np.einsum("ejb,ekja->ekba", Ss, X)  # S_s^T along j
        X = np.einsum("ekc,ekba->ecba", St, X)  # S_t^T along k
        den = (self.lam[:, 2][:, :, None, None] + self.lam[:, 1][:, None, :, None]
               + self.lam[:, 0][:, None, None, :])
        X = X / den
        X = np.einsum("eic,ecba->eiba", St, X)
        X = np.einsum("ejb,eiba->eija", Ss, X)
        X = np.einsum("eka,eija->eijk", Sr, X)
        return X.reshape(E, -1)

    def apply(self, r):
        """z = sum_e R_e^T A~_e^{-1} R_e r on free vectors."""
        m = self.ext >= 0
        rbox = np.where(m, r[np.where(m, self.ext, 0)], 0.0)
        zbox = self.local_solve(rbox)
        return np.bincount(self.ext[m], weights=zbox[m], minlength=r.size)

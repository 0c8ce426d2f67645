"""O5/O6: direct-stiffness summation, restriction, explicit matrices.

Test infrastructure only (see the package docstring).

Q maps unique global values to local copies (v_L = v[gid]); Q^T sums local
copies into unique nodes (np.bincount); R keeps the free (non-Dirichlet)
unique nodes.  The assembled operator is A = R Q^T A_L Q R^T and the
gather-scatter of the method (direct-stiffness summation, the surface
exchange of Sec. 2.2) is v_L <- Q Q^T v_L.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .operator import local_apply


class Numbering:
    """Unique and free numbering of a mesh given by its global ids."""

    def __init__(self, gid: np.ndarray, dirichlet: np.ndarray | None = None):
        self.shape = gid.shape
        uniq, inv = np.unique(gid.ravel(), return_inverse=True)
        self.gids = uniq
        self.n = uniq.size
        self.lid = inv.reshape(gid.shape)  # local -> unique index 0..n-1
        self.mult = np.bincount(self.lid.ravel(), minlength=self.n).astype(np.float64)
        dir_u = np.zeros(self.n, dtype=bool)
        if dirichlet is not None:
            dl = dirichlet.astype(bool)
            cnt = np.bincount(self.lid.ravel(), weights=dl.ravel().astype(float), minlength=self.n)
            if np.any((cnt > 0) & (cnt < self.mult)):
                raise ValueError("Dirichlet flag differs between copies of a node")
            dir_u = cnt > 0
        self.dirichlet_u = dir_u
        self.free = np.flatnonzero(~dir_u)
        self.n_free = self.free.size

    # Q, Q^T, R, R^T
    def Q(self, vu: np.ndarray) -> np.ndarray:
        return vu[self.lid]

    def Qt(self, vl: np.ndarray) -> np.ndarray:
        return np.bincount(self.lid.ravel(), weights=vl.ravel(), minlength=self.n)

    def R(self, vu: np.ndarray) -> np.ndarray:
        return vu[self.free]

    def Rt(self, vf: np.ndarray) -> np.ndarray:
        vu = np.zeros(self.n)
        vu[self.free] = vf
        return vu

    def gs(self, vl: np.ndarray) -> np.ndarray:
        """Direct-stiffness summation Q Q^T v."""
        return self.Q(self.Qt(vl))

    def mask(self, vl: np.ndarray) -> np.ndarray:
        """Zero every local copy of a Dirichlet node."""
        out = vl.copy()
        out[self.dirichlet_u[self.lid]] = 0.0
        return out

    def to_local(self, vf: np.ndarray) -> np.ndarray:
        return self.Q(self.Rt(vf))

    def from_local_consistent(self, vl: np.ndarray) -> np.ndarray:
        """Free unique values of a copy-consistent local vector (mean of copies)."""
        return self.R(self.Qt(vl) / self.mult)


def element_matrices(G, B, N, k=None, h2=0.0) -> np.ndarray:
    """Dense A_e (E, P, P) built column by column from unit vectors."""
    E = G.shape[0]
    P = (N + 1) ** 3
    A = np.empty((E, P, P))
    for q in range(P):
        u = np.zeros((E, P))
        u[:, q] = 1.0
        A[:, :, q] = local_apply(u, G, B, N, k=k, h2=h2)
    return A


def explicit_matrix(G, B, N, num: Numbering, k=None, h2=0.0, free_only=True) -> sp.csr_matrix:
    """Assembled sparse matrix R Q^T A_L Q R^T (or Q^T A_L Q if not free_only)."""
    Ae = element_matrices(G, B, N, k=k, h2=h2)
    E, P, _ = Ae.shape
    rows = np.repeat(num.lid[:, :, None], P, axis=2).ravel()
    cols = np.repeat(num.lid[:, None, :], P, axis=1).ravel()
    A = sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(num.n, num.n)).tocsr()
    if free_only:
        A = A[num.free][:, num.free]
    return A

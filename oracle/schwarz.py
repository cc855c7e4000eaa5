"""Restricted additive Schwarz on one level (oracle; test infrastructure only).

Section 2.2 of the paper: the unknowns are split into np non-overlapping
subdomains, each extended by delta layers of elements; the local matrices
are the principal submatrices J_p = R_p^delta J (R_p^delta)^T and

    B^{-1} = sum_p (R_p^0)^T  J_p^{-1}  R_p^delta

(restricted additive Schwarz: solve on the overlapping subdomain, keep only
the owned part of the local solution).

Partition reading: the paper splits elements and does not name the
partitioner.  Here the interior vertices (the unknowns) are split by
recursive coordinate bisection: at depth d the axis is d mod 3, vertices are
ordered by (coordinate, vertex id), the first floor(|S|/2) go to the lower
half, which gets the lower part ids; the recursion stops at np parts (np a
power of two).  Each interior vertex is owned by exactly one part.  One
layer of overlap adds every interior vertex that shares a tetrahedron with an
owned vertex (the vertices of the layer of elements touching the owned set);
delta layers repeat this.  Dirichlet vertices never enter a subdomain.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import ilu


def rcb(points: np.ndarray, ids: np.ndarray, nparts: int, depth: int = 0):
    """Recursive coordinate bisection; returns a list of id arrays, in part
    order."""
    if nparts <= 1:
        return [np.sort(ids)]
    if nparts & (nparts - 1):
        raise ValueError("nparts must be a power of two")
    ax = depth % 3
    order = np.lexsort((ids, points[:, ax]))  # by coordinate, ties by id
    half = ids.shape[0] // 2
    lo, hi = order[:half], order[half:]
    return rcb(points[lo], ids[lo], nparts // 2, depth + 1) + rcb(points[hi], ids[hi], nparts // 2, depth + 1)


def vertex_graph(nv: int, tets: np.ndarray) -> sp.csr_matrix:
    """Boolean vertex adjacency through shared tetrahedra (with the diagonal)."""
    r = np.repeat(tets, 4, axis=1).ravel()
    c = np.tile(tets, (1, 4)).ravel()
    G = sp.coo_matrix((np.ones(r.size, dtype=np.int8), (r, c)), shape=(nv, nv)).tocsr()
    G.sum_duplicates()
    G.data[:] = 1
    return G


def partition(mesh, nparts: int, overlap: int = 1):
    """Owned sets and overlapping sets S_p (ascending global ids)."""
    interior = np.nonzero(mesh.dirichlet == 0)[0]
    owned = rcb(mesh.xyz[interior], interior, nparts)
    G = vertex_graph(mesh.nv, mesh.tets)
    is_int = mesh.dirichlet == 0
    sets = []
    for own in owned:
        mark = np.zeros(mesh.nv, dtype=bool)
        mark[own] = True
        for _ in range(overlap):
            mark = (G @ mark.astype(np.int8)) > 0
            mark &= is_int
        sets.append(np.nonzero(mark)[0])
    return owned, sets


class RAS:
    """B^{-1} r = sum_p (R^0_p)^T (A[S_p,S_p])^{-1} r[S_p], with LAPACK LU
    (partial pivoting) as the exact subdomain solver, or with ILU(ilu_fill)
    of A[S_p,S_p] (natural ordering) in place of the exact solve (Section 4
    runs the smoother with ILU(p) subdomain solvers)."""

    def __init__(self, A: sp.csr_matrix, dmask: np.ndarray, owned, sets, ilu_fill=None):
        self.dmask = dmask.astype(bool)
        self.owned = owned
        self.sets = sets
        self.ilu_fill = ilu_fill
        self.lu = []
        self.pos = []
        Ad = A.tocsr()
        for own, S in zip(owned, sets):
            if ilu_fill is None:
                self.lu.append(sla.lu_factor(Ad[S][:, S].toarray()))
            else:
                self.lu.append(ilu.ILU(Ad[S][:, S].tocsr(), ilu_fill))
            self.pos.append(np.searchsorted(S, own))

    def apply(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros_like(r)
        z[self.dmask] = r[self.dmask]  # identity rows of the eliminated boundary
        for lu, S, own, pos in zip(self.lu, self.sets, self.owned, self.pos):
            y = sla.lu_solve(lu, r[S]) if self.ilu_fill is None else lu.solve(r[S])
            z[own] = y[pos]
        return z

    def dense(self, n: int) -> np.ndarray:
        """Explicit B^{-1} (tiny problems only)."""
        return np.stack([self.apply(e) for e in np.eye(n)], axis=1)

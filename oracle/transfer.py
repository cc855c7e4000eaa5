"""Barycentric interpolation between independently meshed levels (oracle;
test infrastructure only).

The paper moves vectors between non-nested levels with an interpolation
operator I from one mesh to another (Section 3.2, Figure 6).  Here the
coarse-to-fine operator P_l evaluates the coarse P1 function at every fine
vertex: the vertex is located in a coarse tetrahedron and the coarse nodal
values are combined with its barycentric coordinates
lambda = J^{-1}(x - x0), lambda_0 = 1 - sum(lambda).  The fine-to-coarse
operator is P_l^T.

Location rule: among all coarse tetrahedra with min(lambda) >= -1e-12 the one
with the lowest index wins; if there is none, the tetrahedron with the
largest min(lambda) is used, and a point whose best min(lambda) is below
-1e-8 is an error (it lies outside the coarse mesh).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

ACCEPT = -1e-12
REJECT = -1e-8


class PointLocationError(ValueError):
    pass


def _affine(coarse_xyz, coarse_tets):
    X = coarse_xyz[coarse_tets]
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    return X[:, 0, :], np.linalg.inv(J)


def _bary(x0, Jinv, pts):
    """Barycentric coordinates of pts[k] in tetrahedra t[k]: [k,4]."""
    l123 = np.einsum("kij,kj->ki", Jinv, pts - x0)
    return np.concatenate([1.0 - l123.sum(axis=1, keepdims=True), l123], axis=1)


def locate_bruteforce(coarse_xyz, coarse_tets, pts):
    """Check every point against every tetrahedron (tiny meshes only)."""
    x0, Jinv = _affine(coarse_xyz, coarse_tets)
    nt = coarse_tets.shape[0]
    tet = np.empty(pts.shape[0], dtype=np.int64)
    lam = np.empty((pts.shape[0], 4))
    for k, p in enumerate(pts):
        L = _bary(x0, Jinv, np.repeat(p[None, :], nt, axis=0))
        mn = L.min(axis=1)
        ok = np.nonzero(mn >= ACCEPT)[0]
        t = ok[0] if ok.size else int(np.argmax(mn))
        if mn[t] < REJECT:
            raise PointLocationError(f"point {k} outside the coarse mesh")
        tet[k] = t
        lam[k] = L[t]
    return tet, lam


def locate_bucket(coarse_xyz, coarse_tets, pts, cells_per_tet: float = 1.0):
    """Same rule as locate_bruteforce, with candidates taken from a uniform
    bucket grid over the coarse tetrahedra's (slightly padded) bounding
    boxes."""
    x0, Jinv = _affine(coarse_xyz, coarse_tets)
    nt = coarse_tets.shape[0]
    X = coarse_xyz[coarse_tets]
    lo_all = coarse_xyz.min(axis=0)
    hi_all = coarse_xyz.max(axis=0)
    span = hi_all - lo_all
    nb = max(1, int(round((nt / cells_per_tet) ** (1.0 / 3.0))))
    cell = span / nb
    pad = 1e-9 * span.max()
    bl = np.clip(np.floor((X.min(axis=1) - pad - lo_all) / cell).astype(np.int64), 0, nb - 1)
    bh = np.clip(np.floor((X.max(axis=1) + pad - lo_all) / cell).astype(np.int64), 0, nb - 1)
    # enumerate (bucket, tet) pairs
    pairs_b, pairs_t = [], []
    for t in range(nt):
        r = [np.arange(bl[t, a], bh[t, a] + 1) for a in range(3)]
        g = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
        pairs_b.append(g[:, 0] + nb * (g[:, 1] + nb * g[:, 2]))
        pairs_t.append(np.full(g.shape[0], t))
    pb = np.concatenate(pairs_b)
    pt = np.concatenate(pairs_t)
    order = np.lexsort((pt, pb))
    pb, pt = pb[order], pt[order]
    start = np.searchsorted(pb, np.arange(nb ** 3 + 1))
    q = np.clip(np.floor((pts - lo_all) / cell).astype(np.int64), 0, nb - 1)
    qb = q[:, 0] + nb * (q[:, 1] + nb * q[:, 2])
    tet = np.full(pts.shape[0], -1, dtype=np.int64)
    lam = np.zeros((pts.shape[0], 4))
    best = np.full(pts.shape[0], -np.inf)
    # process candidates in rounds: the r-th candidate of every point
    cnt = start[qb + 1] - start[qb]
    accepted = np.zeros(pts.shape[0], dtype=bool)
    for r in range(int(cnt.max()) if cnt.size else 0):
        act = np.nonzero((cnt > r) & ~accepted)[0]
        if act.size == 0:
            break
        t = pt[start[qb[act]] + r]
        L = _bary(x0[t], Jinv[t], pts[act])
        mn = L.min(axis=1)
        better = mn > best[act]
        acc = mn >= ACCEPT
        upd = acc | better
        tet[act[upd]] = t[upd]
        lam[act[upd]] = L[upd]
        best[act[upd]] = np.where(acc[upd], np.inf, mn[upd])
        accepted[act[acc]] = True
    bad = ~accepted & (best < REJECT)
    if np.any(bad) or np.any(tet < 0):
        raise PointLocationError(f"{int(np.sum(bad | (tet < 0)))} points outside the coarse mesh")
    return tet, lam


def interpolation(fine, coarse, mask_dirichlet: bool = True, locate=locate_bucket) -> sp.csr_matrix:
    """P_l : coarse nodal values -> fine nodal values, shape [nv_f, nv_c].

    With mask_dirichlet, rows of fine Dirichlet vertices are empty (they are
    not located at all) and columns of coarse Dirichlet vertices are zeroed,
    so that the homogeneous boundary condition is kept by the transfer.
    """
    nf, nc = fine.nv, coarse.nv
    rows = np.arange(nf)
    if mask_dirichlet:
        rows = np.nonzero(fine.dirichlet == 0)[0]
    tet, lam = locate(coarse.xyz, coarse.tets, fine.xyz[rows])
    cols = coarse.tets[tet]  # [k,4]
    vals = lam.copy()
    if mask_dirichlet:
        vals[coarse.dirichlet[cols] != 0] = 0.0
    P = sp.coo_matrix((vals.ravel(), (np.repeat(rows, 4), cols.ravel())), shape=(nf, nc)).tocsr()
    P.sum_duplicates()
    return P

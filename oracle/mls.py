"""Overlapping moving-least-squares (MLS) interpolation between non-nested
meshes (oracle; test infrastructure only).

Section 3.2 of the paper.  A value at a target node x* is interpolated from
the source nodes x~_n of the neighbourhood N(x*) = { x~_n : |x~_n - x*| <
rho(x*) } by minimising the weighted loss

    L(a) = sum_n w(x* - x~_n) [p(x~_n)^T a - u~_n]^2,
    w = 1 - 6 r^2 + 8 r^3 - 3 r^4,   r = |x* - x~_n| / rho(x*),

over the coefficients a of the polynomial space with basis p.  Its
stationary point solves P1 a = P2 u~ with P1 = P D P^T, P2 = P D, where the
columns of P are p(x~_n) and D = diag(w) (Theorem 1: unique when
rank(P) = |P|).  The interpolated value is u* = p(x*)^T P1^{-1} P2 u~, so the
row of the operator for x* is phi = p(x*)^T P1^{-1} P2, and stacking the rows
of every target node gives the operator (equation *interpolation f*).

Readings where the paper leaves a choice open (the library takes the same):
  * the polynomial space is linear, p(x) = [1, x, y, z] (|P| = 4), the space
    of the P1 unknowns;
  * the scale starts at rho_0 = alpha * h, h = the mean edge length of the
    source mesh, alpha = 1.0 by default, and grows by the factor 1.25 until
    rank(P) = 4 (the paper grows rho until the rank is full);
  * rank(P) = 4 is decided on the centred, rho-scaled basis
    [1, (x - x*) / rho] (the same space): its smallest singular value must
    exceed 1e-6 times its largest;
  * by default the neighbourhood is not clipped: on one device the whole
    source level is local.  With `clip` it is the paper's
    N~(x*) = {x~_n in Omega~^delta_p : |x~_n - x*| < rho(x*)}: processor p
    owns the target node (its subdomain on the target level), and its
    overlapping subdomain of the source level is the source level's own
    coordinate bisection into the same number of parts (every level is split
    across the same processors, Section 3.1), extended by delta layers, as
    the nodes of the elements that touch it (`clip_sets`);
  * homogeneous Dirichlet conditions: rows of Dirichlet target nodes are
    empty and the weights of Dirichlet source nodes are dropped after the
    solve (as for the barycentric transfer).

The coarse-to-fine operator P_l is this interpolation from coarse (source)
to fine (target) nodes; the fine-to-coarse transfer used by the V-cycle is
its transpose.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

ALPHA = 1.0
GROWTH = 1.25
RANK_TOL = 1e-6


def weight(r):
    """w as a function of r = distance / rho (the loss of Section 3.2)."""
    r = np.asarray(r, dtype=np.float64)
    return 1.0 - 6.0 * r ** 2 + 8.0 * r ** 3 - 3.0 * r ** 4


def basis(x):
    """Linear basis p(x) = [1, x, y, z] as columns: shape [4, m]."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    return np.vstack([np.ones(len(x)), x.T])


def mean_edge_length(xyz, tets) -> float:
    """Mean length of the distinct edges of a tetrahedral mesh."""
    pairs = np.array([(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)])
    e = np.sort(tets[:, pairs].reshape(-1, 2), axis=1)
    e = np.unique(e, axis=0)
    return float(np.linalg.norm(xyz[e[:, 0]] - xyz[e[:, 1]], axis=1).mean())


def full_rank(xstar, pts, rho) -> bool:
    """rank(P) = |P| for the neighbours pts of xstar (Theorem 1's condition)."""
    if len(pts) < 4:
        return False
    Q = basis((pts - xstar) / rho)
    s = np.linalg.svd(Q, compute_uv=False)
    return bool(s[-1] > RANK_TOL * s[0])


def mls_row(xstar, pts, rho):
    """phi = p(x*)^T P1^{-1} P2 for the neighbours pts (all within rho)."""
    r = np.linalg.norm(pts - xstar, axis=1) / rho
    D = np.diag(weight(r))
    P = basis(pts)
    P1 = P @ D @ P.T
    P2 = P @ D
    return basis(xstar)[:, 0] @ np.linalg.solve(P1, P2)


def neighbourhood(tree, src_xyz, xstar, rho0, allowed=None):
    """(ids, rho): source nodes strictly within rho of x* (and in `allowed`, a
    boolean mask, when given), rho grown from rho0 by GROWTH until the
    neighbourhood has full rank."""
    rho = rho0
    for _ in range(200):
        ids = np.array(sorted(tree.query_ball_point(xstar, rho)), dtype=np.int64)
        if len(ids):
            ids = ids[np.linalg.norm(src_xyz[ids] - xstar, axis=1) < rho]
        if allowed is not None and len(ids):
            ids = ids[allowed[ids]]
        if full_rank(xstar, src_xyz[ids], rho):
            return ids, rho
        rho *= GROWTH
    raise ValueError("no full-rank neighbourhood")


def clip_sets(target, source, nparts: int, overlap: int = 1):
    """(owner of every target node, boolean masks of the source nodes of every
    processor): the target level's partition into nparts and the source
    level's own partition into the same nparts, extended by `overlap` layers,
    taken as the nodes of the source elements touching it (its subdomain
    Omega~^delta_p, boundary nodes included)."""
    from . import schwarz

    owned_t, _ = schwarz.partition(target, nparts, overlap)
    owner = -np.ones(target.nv, dtype=np.int64)
    for p, o in enumerate(owned_t):
        owner[o] = p
    _, sets_s = schwarz.partition(source, nparts, overlap)
    masks = []
    for S in sets_s:
        inset = np.zeros(source.nv, dtype=bool)
        inset[S] = True
        touch = inset[source.tets].any(axis=1)
        m = np.zeros(source.nv, dtype=bool)
        m[source.tets[touch].ravel()] = True
        masks.append(m)
    return owner, masks


def interpolation(target, source, alpha: float = ALPHA, mask_dirichlet: bool = True, rows=None,
                  clip=None) -> sp.csr_matrix:
    """MLS operator from source nodal values to target nodal values, shape
    [target.nv, source.nv].  rows: optional subset of target nodes to build
    (the other rows stay empty).  clip: None, or (owner, masks) of
    clip_sets -- the neighbourhood of a target node owned by p is clipped to
    masks[p] (nodes without an owner, Dirichlet ones, are not clipped)."""
    h = mean_edge_length(source.xyz, source.tets)
    tree = cKDTree(source.xyz)
    if rows is None:
        rows = np.arange(target.nv)
    ri, ci, vi = [], [], []
    for v in rows:
        if mask_dirichlet and target.dirichlet[v]:
            continue
        xs = target.xyz[v]
        allowed = None if clip is None or clip[0][v] < 0 else clip[1][clip[0][v]]
        ids, rho = neighbourhood(tree, source.xyz, xs, alpha * h, allowed)
        phi = mls_row(xs, source.xyz[ids], rho)
        if mask_dirichlet:
            keep = source.dirichlet[ids] == 0
            ids, phi = ids[keep], phi[keep]
        ri.append(np.full(len(ids), v))
        ci.append(ids)
        vi.append(phi)
    if ri:
        ri, ci, vi = np.concatenate(ri), np.concatenate(ci), np.concatenate(vi)
    return sp.csr_matrix((vi, (ri, ci)), shape=(target.nv, source.nv))


def prolongation(fine, coarse, alpha: float = ALPHA, mask_dirichlet: bool = True, clip_parts: int = 0,
                 overlap: int = 1) -> sp.csr_matrix:
    """P_l: coarse -> fine by MLS (the coarse nodes are the sources);
    clip_parts > 0 clips every neighbourhood to the target's processor's
    coarse subdomain (clip_sets)."""
    clip = clip_sets(fine, coarse, clip_parts, overlap) if clip_parts else None
    return interpolation(fine, coarse, alpha, mask_dirichlet, clip=clip)


def restriction(fine, coarse, alpha: float = ALPHA, mask_dirichlet: bool = True, clip_parts: int = 0,
                overlap: int = 1) -> sp.csr_matrix:
    """R_l: fine -> coarse by MLS (the fine nodes are the sources; the scale
    starts at alpha times the fine mesh's mean edge length): the paper's
    second interpolation, applied to the residual as it stands."""
    clip = clip_sets(coarse, fine, clip_parts, overlap) if clip_parts else None
    return interpolation(coarse, fine, alpha, mask_dirichlet, clip=clip)

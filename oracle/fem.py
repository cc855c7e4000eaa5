"""P1 finite elements on tetrahedra (oracle; test infrastructure only).

The paper writes the discrete problem as J_M u_M = b_M with b = -Psi(0) and
J the Jacobian of the discrete residual Psi (Section 2.1, equation
'discretized').  For the linear problem -div(kappa grad u) = f with
homogeneous Dirichlet data the Jacobian is the P1 stiffness matrix and b the
load vector.  The element-wise formulas below are the textbook ones:
  |T| = |det J| / 6 with J = [x1-x0, x2-x0, x3-x0],
  grad lambda_{1..3} = rows of J^{-1}, grad lambda_0 = -sum of the others,
  K_ab = kappa_T |T| grad lambda_a . grad lambda_b,  kappa_T = kappa(centroid).
"""
from __future__ import annotations

from itertools import combinations_with_replacement
from math import factorial

import numpy as np
import scipy.sparse as sp


def tet_geometry(xyz: np.ndarray, tets: np.ndarray):
    """Signed volumes, barycentric gradients [nt,4,3] and centroids of every
    tetrahedron."""
    X = xyz[tets]  # [nt,4,3]
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))  # columns are edges
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    g = np.empty((tets.shape[0], 4, 3))
    g[:, 1:, :] = Jinv  # row a of J^{-1} is grad lambda_a
    g[:, 0, :] = -Jinv.sum(axis=1)
    return det / 6.0, g, X.mean(axis=1)


def check_mesh(xyz, tets):
    """All signed volumes must be positive (a bad mesh is an error)."""
    vol, _, _ = tet_geometry(xyz, tets)
    if np.any(vol <= 0):
        raise ValueError("non-positive tetrahedron volume")
    return vol


def kappa_eval(points: np.ndarray, kappa) -> np.ndarray:
    """kappa at points: constant, or exp(sum_k mu_k exp(-|x-c_k|^2/width))."""
    if kappa.kind == "const":
        return np.full(points.shape[0], float(kappa.value))
    if kappa.kind == "loggauss":
        d2 = ((points[:, None, :] - kappa.centres[None, :, :]) ** 2).sum(axis=2)
        return np.exp((kappa.mu[None, :] * np.exp(-d2 / kappa.width)).sum(axis=1))
    if kappa.kind == "per_tet":
        return np.asarray(kappa.value, dtype=np.float64)
    raise ValueError(kappa.kind)


def stiffness_neumann(xyz, tets, kappa) -> sp.csr_matrix:
    """Unconstrained P1 stiffness matrix A_N = sum_T kappa_T |T| G_T G_T^T."""
    vol, g, cen = tet_geometry(xyz, tets)
    kT = kappa_eval(cen, kappa)
    Ke = np.einsum("t,tai,tbi->tab", kT * np.abs(vol), g, g)
    rows = np.repeat(tets, 4, axis=1).ravel()
    cols = np.tile(tets, (1, 4)).ravel()
    n = xyz.shape[0]
    A = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def load_const(xyz, tets, f: float = 1.0) -> np.ndarray:
    """Load vector of a constant f: every vertex of T receives f |T| / 4."""
    vol, _, _ = tet_geometry(xyz, tets)
    b = np.zeros(xyz.shape[0])
    np.add.at(b, tets.ravel(), np.repeat(f * np.abs(vol) / 4.0, 4))
    return b


def load_per_tet(xyz, tets, fT: np.ndarray) -> np.ndarray:
    """Load vector of an f constant on every tetrahedron (values fT[nt]):
    b_a = sum over the tetrahedra T at a of f_T |T| / 4, the exact integral
    of f lambda_a (int_T lambda_a = |T| / 4)."""
    vol, _, _ = tet_geometry(xyz, tets)
    b = np.zeros(xyz.shape[0])
    np.add.at(b, tets.ravel(), np.repeat(np.asarray(fT, dtype=np.float64) * np.abs(vol) / 4.0, 4))
    return b


def load_nodal(xyz, tets, fv: np.ndarray) -> np.ndarray:
    """Load vector of the P1 interpolant f_h = sum_j f_j phi_j of nodal values
    fv[nv], integrated exactly: b = M f with the P1 mass matrix, whose element
    entries are int_T lambda_a lambda_b = |T| (1 + delta_ab) / 20."""
    vol, _, _ = tet_geometry(xyz, tets)
    fv = np.asarray(fv, dtype=np.float64)
    Me = np.abs(vol)[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None, :, :] / 20.0
    contrib = np.einsum("tab,tb->ta", Me, fv[tets])
    b = np.zeros(xyz.shape[0])
    np.add.at(b, tets.ravel(), contrib.ravel())
    return b


def load(mesh, f) -> np.ndarray:
    """Load vector of a source term: a number (constant f) or a field with
    kind 'per_tet' / 'nodal' and values on this mesh."""
    if isinstance(f, (int, float, np.floating)):
        return load_const(mesh.xyz, mesh.tets, float(f))
    if f.kind == "per_tet":
        return load_per_tet(mesh.xyz, mesh.tets, f.values)
    if f.kind == "nodal":
        return load_nodal(mesh.xyz, mesh.tets, f.values)
    raise ValueError(f.kind)


def grundmann_moeller(s: int, dim: int = 3):
    """Grundmann-Moeller rule of degree 2s+1 on a simplex (SIAM J. Numer.
    Anal. 15, 1978).  Returns barycentric points [q, dim+1] and weights [q]
    that sum to 1 (i.e. weights relative to the simplex volume)."""
    d = 2 * s + 1
    pts, wts = [], []
    for i in range(s + 1):
        w = (-1) ** i * 2.0 ** (-2 * s) * (d + dim - 2 * i) ** d / (factorial(i) * factorial(d + dim - i))
        w *= factorial(dim)  # relative to the simplex volume 1/dim!
        m = s - i
        for combo in combinations_with_replacement(range(dim + 1), m):
            beta = np.zeros(dim + 1)
            for c in combo:
                beta[c] += 1
            pts.append((2 * beta + 1) / (d + dim - 2 * i))
            wts.append(w)
    return np.array(pts), np.array(wts)


def load_quadrature(xyz, tets, f, s: int = 2) -> np.ndarray:
    """Load vector b_a = int f lambda_a by a Grundmann-Moeller rule of degree
    2s+1 (f is a callable on [q,3] points)."""
    vol, _, _ = tet_geometry(xyz, tets)
    lam, w = grundmann_moeller(s)
    X = xyz[tets]  # [nt,4,3]
    b = np.zeros(xyz.shape[0])
    for q in range(lam.shape[0]):
        p = np.einsum("a,tai->ti", lam[q], X)
        fv = f(p) * np.abs(vol) * w[q]
        np.add.at(b, tets.ravel(), (fv[:, None] * lam[q][None, :]).ravel())
    return b


def l2_error(xyz, tets, x, u, s: int = 2) -> float:
    """|| u - sum_i x_i phi_i ||_{L2} by a Grundmann-Moeller rule."""
    vol, _, _ = tet_geometry(xyz, tets)
    lam, w = grundmann_moeller(s)
    X = xyz[tets]
    xv = x[tets]  # [nt,4]
    err = 0.0
    for q in range(lam.shape[0]):
        p = np.einsum("a,tai->ti", lam[q], X)
        uh = xv @ lam[q]
        err += np.sum(w[q] * np.abs(vol) * (u(p) - uh) ** 2)
    return float(np.sqrt(err))


def dirichlet_eliminate(A_N: sp.csr_matrix, b: np.ndarray, dmask: np.ndarray):
    """Symmetric elimination of homogeneous Dirichlet vertices: rows and
    columns of D are removed from A_N and replaced by the identity, b_D = 0."""
    d = dmask.astype(bool)
    keep = sp.diags((~d).astype(np.float64))
    A = (keep @ A_N @ keep).tocsr() + sp.diags(d.astype(np.float64))
    A = A.tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    bb = b.copy()
    bb[d] = 0.0
    return A, bb


def assemble(mesh, kappa, f=1.0):
    """The Dirichlet-eliminated system (A, b) of one mesh and coefficient; f
    as in `load`."""
    check_mesh(mesh.xyz, mesh.tets)
    A_N = stiffness_neumann(mesh.xyz, mesh.tets, kappa)
    b = load(mesh, f)
    return dirichlet_eliminate(A_N, b, mesh.dirichlet)

"""P1 linear elasticity with the field-split interpolation (oracle; test
infrastructure only).

Section 4.2 of the paper solves linear elasticity, -div sigma = f, with the
stress sigma = lambda tr(eps) I + 2 mu eps of the strain eps = (grad u +
grad u^T) / 2 and the Lame coefficients of Young's modulus E and Poisson's
ratio nu: mu = E / (2 (1 + nu)), lambda = E nu / ((1 + nu)(1 - 2 nu)).  Here
the displacement is P1 on tetrahedra (three unknowns per vertex, numbered
3 v + c for component c of vertex v), E is constant on every tetrahedron (a
kappa-type field, E_T = kappa_T), all three components vanish on the
Dirichlet vertices, and f is a body force.

Section 3.2 moves a multi-field vector between levels by splitting its
unknowns into fields that have at most one unknown per node (equation
field-split) and interpolating every field with an operator of its own
(equation interpolation split): I = sum_f R_f^T I^f R~_f, R_f extracting the
unknowns of field f.  The three displacement components live on the same P1
nodes, so each field uses the scalar transfer P_l of the mesh pair.

The element matrix is the textbook Voigt form K_T = |T| B^T D B with the
engineering strains (e_xx, e_yy, e_zz, g_yz, g_xz, g_xy) = B u_T and the
isotropic stiffness D.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem, krylov, multilevel, schwarz, transfer
from .problem import OracleHierarchy, level_kappa

NCOMP = 3


def lame(E, nu):
    """(mu, lambda) of Young's modulus and Poisson's ratio."""
    E = np.asarray(E, dtype=np.float64)
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def voigt_stiffness(E: float, nu: float) -> np.ndarray:
    """6x6 isotropic D with sigma_voigt = D eps_voigt (engineering shears)."""
    mu, lam = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] = lam + 2.0 * mu
    D[np.arange(3, 6), np.arange(3, 6)] = mu
    return D


def strain_matrix(g: np.ndarray) -> np.ndarray:
    """6x12 B of one tetrahedron from its barycentric gradients g[4,3]:
    column 3a + c is the displacement of vertex a in direction c."""
    B = np.zeros((6, 12))
    for a in range(4):
        gx, gy, gz = g[a]
        B[0, 3 * a + 0] = gx
        B[1, 3 * a + 1] = gy
        B[2, 3 * a + 2] = gz
        B[3, 3 * a + 1], B[3, 3 * a + 2] = gz, gy  # g_yz = du_y/dz + du_z/dy
        B[4, 3 * a + 0], B[4, 3 * a + 2] = gz, gx  # g_xz
        B[5, 3 * a + 0], B[5, 3 * a + 1] = gy, gx  # g_xy
    return B


def dofs_of(tets: np.ndarray) -> np.ndarray:
    """[nt,12] unknowns of every tetrahedron, 3 a + c order."""
    return (NCOMP * np.repeat(tets, NCOMP, axis=1) + np.tile(np.arange(NCOMP), 4)[None, :]).astype(np.int64)


def stiffness_neumann(xyz, tets, E_T, nu: float) -> sp.csr_matrix:
    """Unconstrained elasticity matrix sum_T |T| B_T^T D(E_T) B_T (3nv x 3nv)."""
    vol, g, _ = fem.tet_geometry(xyz, tets)
    E_T = np.broadcast_to(np.asarray(E_T, dtype=np.float64), (tets.shape[0],))
    Ke = np.empty((tets.shape[0], 12, 12))
    for t in range(tets.shape[0]):
        B = strain_matrix(g[t])
        Ke[t] = abs(vol[t]) * (B.T @ voigt_stiffness(E_T[t], nu) @ B)
    d = dofs_of(tets)
    rows = np.repeat(d, 12, axis=1).ravel()
    cols = np.tile(d, (1, 12)).ravel()
    n = NCOMP * xyz.shape[0]
    A = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def load(mesh, f) -> np.ndarray:
    """Load vector of a body force: a 3-vector (constant), or a field of kind
    'per_tet' (values [nt,3]) or 'nodal' (values [nv,3]); every component is
    the scalar load of that component (fem.load)."""
    b = np.zeros(NCOMP * mesh.nv)
    if np.ndim(f) == 1 and len(f) == NCOMP and not hasattr(f, "kind"):
        for c in range(NCOMP):
            b[c::NCOMP] = fem.load_const(mesh.xyz, mesh.tets, float(f[c]))
        return b
    vals = np.asarray(f.values, dtype=np.float64).reshape(-1, NCOMP)
    for c in range(NCOMP):
        b[c::NCOMP] = fem.load(mesh, type(f)(f.kind, vals[:, c].copy()))
    return b


def dof_mask(dirichlet: np.ndarray) -> np.ndarray:
    return np.repeat(np.asarray(dirichlet), NCOMP)


def assemble(mesh, E_field, nu: float, f=(0.0, 0.0, -1.0)):
    """Dirichlet-eliminated (A, b) of one mesh: E_T from the kappa-type field
    at the centroids (or given per tetrahedron)."""
    fem.check_mesh(mesh.xyz, mesh.tets)
    _, _, cen = fem.tet_geometry(mesh.xyz, mesh.tets)
    E_T = fem.kappa_eval(cen, E_field)
    A_N = stiffness_neumann(mesh.xyz, mesh.tets, E_T, nu)
    return fem.dirichlet_eliminate(A_N, load(mesh, f), dof_mask(mesh.dirichlet))


def field_selector(n_nodes: int, c: int) -> sp.csr_matrix:
    """R_c: the unknowns of field (component) c out of the interleaved vector."""
    rows = np.arange(n_nodes)
    return sp.csr_matrix((np.ones(n_nodes), (rows, NCOMP * rows + c)), shape=(n_nodes, NCOMP * n_nodes))


def split_interpolation(P: sp.csr_matrix) -> sp.csr_matrix:
    """I = sum_f R_f^T P R~_f (equation interpolation split), every field
    interpolated by the scalar P from the coarse to the fine nodes."""
    nf, nc = P.shape
    I = sp.csr_matrix((NCOMP * nf, NCOMP * nc))
    for c in range(NCOMP):
        I = I + field_selector(nf, c).T @ P @ field_selector(nc, c)
    return I.tocsr()


def expand_sets(owned, sets):
    """Subdomains of vertices -> subdomains of their unknowns (ascending)."""
    ex = lambda v: (NCOMP * np.asarray(v)[:, None] + np.arange(NCOMP)[None, :]).ravel()
    return [ex(o) for o in owned], [ex(s) for s in sets]


def build(problem, nu: float = 0.3, f=(0.0, 0.0, -1.0), locate=transfer.locate_bucket) -> OracleHierarchy:
    """The elasticity hierarchy of a workload: every level rediscretised with
    E from the problem's kappa field, partitions of the vertices (the scalar
    rule) carried to their unknowns, split barycentric transfers, the V-cycle
    of Algorithm 2 with exact subdomain solves."""
    meshes = problem.meshes
    L = len(meshes)
    A, P, parts, levels = [], [], [], []
    b = None
    for l, m in enumerate(meshes):
        Al, bl = assemble(m, level_kappa(problem.kappa, l), nu, f if l == 0 else (0.0, 0.0, 0.0))
        A.append(Al)
        if l == 0:
            b = bl
    for l in range(L - 1):
        P.append(split_interpolation(transfer.interpolation(meshes[l], meshes[l + 1], locate=locate)))
        owned, sets = expand_sets(*schwarz.partition(meshes[l], problem.nparts[l], problem.overlap))
        parts.append((owned, sets))
        ras = schwarz.RAS(A[l], dof_mask(meshes[l].dirichlet), owned, sets)
        levels.append(multilevel.Level(A[l], dof_mask(meshes[l].dirichlet), ras, P[l]))
    levels.append(multilevel.Level(A[L - 1], dof_mask(meshes[L - 1].dirichlet)))
    return OracleHierarchy(problem, A, b, P, parts, multilevel.VCycle(levels, problem.its))


def rigid_modes(xyz: np.ndarray) -> np.ndarray:
    """The six rigid motions (three translations, three rotations) as
    interleaved vectors [6, 3nv]."""
    nv = xyz.shape[0]
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    o, i = np.zeros(nv), np.ones(nv)
    fields = [(i, o, o), (o, i, o), (o, o, i), (-y, x, o), (o, -z, y), (z, o, -x)]
    return np.array([np.stack(f, axis=1).ravel() for f in fields])

"""Whole-hierarchy oracle: assemble every level, build transfers, smoothers
and the V-cycle, then solve with FGMRES (test infrastructure only).

Input: a ``workloads.Problem`` (meshes fine..coarse, subdomain counts per
smoothed level, kappa).  The finest level carries the system the outer
Krylov method solves; coarser levels are rediscretised with kappa at their
own centroids (the Jacobian each level provides in Algorithm 2).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.sparse.linalg as spla

from . import fem, krylov, mls, multilevel, schwarz, transfer


@dataclass
class OracleHierarchy:
    problem: object
    A: List  # per level, Dirichlet-eliminated CSR
    b: np.ndarray  # fine load vector (f = 1)
    P: List  # P[l] maps level l+1 -> l
    parts: List  # (owned, sets) per smoothed level
    vcycle: multilevel.VCycle


def level_kappa(kappa, l: int):
    """The coefficient of level l: per-tetrahedron values come as one array
    per level, any other kind is a field of the whole domain."""
    if getattr(kappa, "kind", None) == "per_tet" and isinstance(kappa.value, (list, tuple)):
        return type(kappa)(kind="per_tet", value=kappa.value[l])
    return kappa


def build(problem, f=1.0, locate=transfer.locate_bucket, mls_alpha: Optional[float] = None,
          ilu_fill: Optional[List[int]] = None, mls_restrict: bool = False,
          mls_clip: bool = False) -> OracleHierarchy:
    """f: the source term of the finest level's load (a number, or a field of
    kind 'per_tet' / 'nodal' with values on the finest mesh).
    mls_alpha: None for the barycentric transfer, else the MLS transfer of
    Section 3.2 with initial scale mls_alpha times the coarse mean edge.
    ilu_fill: None for exact subdomain solves, else the ILU fill level of
    every smoothed level (the coarsest level is always solved directly).
    mls_restrict: with the MLS transfer, restrict by the fine-to-coarse MLS
    interpolation instead of P^T.
    mls_clip: with the MLS transfer, clip every neighbourhood to the
    overlapping subdomain of the target's processor (the fine level's
    subdomain count on both levels)."""
    meshes = problem.meshes
    L = len(meshes)
    A, P, parts, levels = [], [], [], []
    b = None
    for l, m in enumerate(meshes):
        Al, bl = fem.assemble(m, level_kappa(problem.kappa, l), f if l == 0 else 1.0)
        A.append(Al)
        if l == 0:
            b = bl
    for l in range(L - 1):
        if mls_alpha is None:
            P.append(transfer.interpolation(meshes[l], meshes[l + 1], locate=locate))
        else:
            clip = problem.nparts[l] if mls_clip else 0
            P.append(mls.prolongation(meshes[l], meshes[l + 1], mls_alpha, clip_parts=clip, overlap=problem.overlap))
        owned, sets = schwarz.partition(meshes[l], problem.nparts[l], problem.overlap)
        parts.append((owned, sets))
        ras = schwarz.RAS(A[l], meshes[l].dirichlet, owned, sets, None if ilu_fill is None else ilu_fill[l])
        R = None
        if mls_restrict and mls_alpha is not None:
            R = mls.restriction(meshes[l], meshes[l + 1], mls_alpha, clip_parts=problem.nparts[l] if mls_clip else 0,
                                overlap=problem.overlap)
        levels.append(multilevel.Level(A[l], meshes[l].dirichlet, ras, P[l], R))
    levels.append(multilevel.Level(A[L - 1], meshes[L - 1].dirichlet))
    vc = multilevel.VCycle(levels, problem.its)
    return OracleHierarchy(problem, A, b, P, parts, vc)


def solve(h: OracleHierarchy, b: Optional[np.ndarray] = None, rtol: Optional[float] = None,
          restart: Optional[int] = None, max_it: int = 1000) -> krylov.FGMRESResult:
    pb = h.problem
    bb = h.b if b is None else b
    return krylov.fgmres(h.A[0], bb, h.vcycle, restart or pb.restart, rtol or pb.rtol, max_it)


def exact(h: OracleHierarchy, b: Optional[np.ndarray] = None) -> np.ndarray:
    """x* = A^{-1} b by a sparse direct solve."""
    bb = h.b if b is None else b
    return spla.splu(h.A[0].tocsc()).solve(bb)

"""Geometry-preserving mesh coarsening, Algorithm 1 (oracle; test
infrastructure only).

Section 3.1 of the paper coarsens M_i into M_{i+1} by repeating, up to M
times: take a maximal independent set S of the graph of the interior
vertices (two vertices adjacent when they share an element), delete the
elements around every vertex of S, and fill each cavity with new elements
from its surface (the paper uses the CPAFT advancing-front mesher, which it
only cites).  Boundary vertices are never removed, so the boundary surface is
kept exactly.

Readings (the library takes the same):
  * interior vertex = non-Dirichlet vertex; boundary = Dirichlet;
  * the MIS is the greedy one in increasing priority, priority(v) =
    splitmix64(seed + 2^40 * round + v) (ties by vertex id), which is also
    what Luby's parallel algorithm returns with these priorities;
  * a cavity is re-meshed by contracting the removed vertex v onto one of
    its neighbours u (the edge-contraction method the paper builds on): the
    elements containing the edge (v, u) disappear, the others of the star
    of v get u in place of v.  Of the neighbours (ascending id) the one
    whose new elements have the largest smallest quality is taken, quality
    q = sqrt(2) * 6V / l_rms^3 (1 for a regular tetrahedron, l_rms the
    root mean square of the six edge lengths); with no neighbour reaching
    q > QMIN the vertex stays (stars of independent vertices are disjoint,
    so the contractions of one round do not interact);
  * vertices keep their positions (no smoothing); the output numbers the
    surviving vertices in ascending old id and keeps the elements in their
    old order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

import numpy as np

QMIN = 0.02
MASK = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One output of the SplitMix64 generator (Steele, Lea, Flood 2014) for state x."""
    z = (x + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def priority(seed: int, rnd: int, v: int) -> int:
    return splitmix64((seed + (rnd << 40) + v) & MASK)


def det6(p0, p1, p2, p3) -> float:
    """6 x the signed volume of (p0, p1, p2, p3), cofactor expansion."""
    a = [p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]]
    b = [p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]]
    c = [p3[0] - p0[0], p3[1] - p0[1], p3[2] - p0[2]]
    return (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0])
            + a[2] * (b[0] * c[1] - b[1] * c[0]))


def quality(p0, p1, p2, p3) -> float:
    pts = (p0, p1, p2, p3)
    s = 0.0
    for i in range(4):
        for j in range(i + 1, 4):
            dx = pts[i][0] - pts[j][0]
            dy = pts[i][1] - pts[j][1]
            dz = pts[i][2] - pts[j][2]
            s += dx * dx + dy * dy + dz * dz
    lr = math.sqrt(s / 6.0)
    return math.sqrt(2.0) * det6(p0, p1, p2, p3) / (lr * lr * lr)


def vertex_neighbours(nv: int, tets: List[List[int]]):
    nb = [set() for _ in range(nv)]
    for t in tets:
        for a in t:
            for b in t:
                if a != b:
                    nb[a].add(b)
    return nb


def mis(nv, tets, alive, boundary, seed, rnd):
    """Greedy maximal independent set of the alive interior vertices in
    increasing priority (ties by id)."""
    nb = vertex_neighbours(nv, tets)
    cand = [v for v in range(nv) if alive[v] and not boundary[v]]
    cand.sort(key=lambda v: (priority(seed, rnd, v), v))
    inS = [False] * nv
    S = []
    for v in cand:
        if not any(inS[w] for w in nb[v]):
            inS[v] = True
            S.append(v)
    return S, nb


@dataclass
class Result:
    xyz: np.ndarray
    tets: np.ndarray
    dirichlet: np.ndarray
    removed: int
    kept_ids: np.ndarray  # old id of every new vertex


def coarsen(xyz, tets, dirichlet, rounds: int, seed: int) -> Result:
    xyz = np.asarray(xyz, dtype=np.float64)
    P = [tuple(p) for p in xyz]
    T = [list(map(int, t)) for t in np.asarray(tets)]
    nv = len(P)
    boundary = [bool(d) for d in np.asarray(dirichlet)]
    alive = [True] * nv
    removed = 0
    for rnd in range(rounds):
        S, nb = mis(nv, [t for t in T if t is not None], alive, boundary, seed, rnd)
        if not S:
            break
        star = {v: [] for v in S}
        for e, t in enumerate(T):
            if t is None:
                continue
            for a in t:
                if a in star:
                    star[a].append(e)
        for v in S:
            best_u, best_q = -1, QMIN
            for u in sorted(nb[v]):
                qmin = math.inf
                for e in star[v]:
                    t = T[e]
                    if u in t:
                        continue
                    nt = [u if a == v else a for a in t]
                    qmin = min(qmin, quality(P[nt[0]], P[nt[1]], P[nt[2]], P[nt[3]]))
                if qmin > best_q:
                    best_u, best_q = u, qmin
            if best_u < 0:
                continue
            for e in star[v]:
                t = T[e]
                T[e] = None if best_u in t else [best_u if a == v else a for a in t]
            alive[v] = False
            removed += 1
    kept = np.array([v for v in range(nv) if alive[v]], dtype=np.int64)
    new_id = -np.ones(nv, dtype=np.int64)
    new_id[kept] = np.arange(len(kept))
    out_t = np.array([[new_id[a] for a in t] for t in T if t is not None], dtype=np.int64)
    return Result(xyz[kept], out_t, np.asarray(dirichlet)[kept].astype(np.uint8), removed, kept)

"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module produces *inputs only*: jittered Kuhn-split cube meshes, the
seeds and draws of the log-Gaussian diffusion coefficient (centres and
amplitudes), right-hand sides and request traces.  It contains none of the
method's arithmetic: no assembly, no coefficient evaluation, no transfer,
partition, smoother or Krylov step.  Both the independent CPU oracle and the
GPU library consume what is generated here.

The paper's own geometries (a lake-shaped 2D domain, a drive wheel, a vessel;
Section 4) are not available; jittered unit-cube meshes of comparable and
larger vertex counts stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations
from typing import List, Optional, Sequence

import numpy as np

JITTER = 0.2  # interior vertices move by U[-0.2h, 0.2h] per coordinate
KAPPA_WIDTH = 0.02  # denominator of the Gaussian bumps in log kappa


@dataclass
class Mesh:
    """A tetrahedral mesh of the unit cube.

    xyz       float64[nv, 3]   vertex coordinates
    tets      int32[nt, 4]     vertex ids, positively oriented on the
                               un-jittered grid
    dirichlet uint8[nv]        1 on the cube faces (homogeneous Dirichlet)
    n         cells per side of the generating grid
    """

    xyz: np.ndarray
    tets: np.ndarray
    dirichlet: np.ndarray
    n: int
    seed: Optional[int] = None

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tets.shape[0])


def _kuhn_cell_pattern():
    """Six tetrahedra of the Kuhn split of a unit cell, as corner offsets.

    For every permutation (a, b, c) of the axes, in lexicographic order, the
    tetrahedron runs from the cell's low corner along e_a, then e_b, then e_c
    to the high corner.  Odd permutations get their middle vertices swapped so
    that every tetrahedron is positively oriented.
    """
    pats = []
    for perm in permutations(range(3)):
        corners = [np.zeros(3, dtype=np.int64)]
        cur = np.zeros(3, dtype=np.int64)
        for ax in perm:
            cur = cur.copy()
            cur[ax] += 1
            corners.append(cur)
        # parity of the permutation
        inv = sum(1 for i in range(3) for j in range(i + 1, 3) if perm[i] > perm[j])
        if inv % 2 == 1:
            corners[1], corners[2] = corners[2], corners[1]
        pats.append(corners)
    return np.array(pats, dtype=np.int64)  # [6, 4, 3]


def kuhn_cube(n: int, seed: Optional[int] = None, jitter: float = JITTER) -> Mesh:
    """Kuhn-split n^3 grid of the unit cube, interior vertices jittered.

    Vertex (i, j, k) has id i + (n+1)(j + (n+1)k) and sits at (i, j, k)/n.
    With a seed, every coordinate of every vertex gets an independent
    U[-jitter*h, jitter*h] draw (PCG64 via numpy's default_rng, all vertices
    in id order, x/y/z interleaved), which is then kept for interior vertices
    only, so the cube faces stay planar and the cube is tiled exactly.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    m = n + 1
    ii, jj, kk = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    # id = i + m*(j + m*k): order vertices with i fastest
    idx = np.stack([ii, jj, kk], axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    xyz = idx.astype(np.float64) * h
    boundary = np.any((idx == 0) | (idx == n), axis=1)
    if seed is not None and jitter > 0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
        d[boundary] = 0.0
        xyz = xyz + d
    pats = _kuhn_cell_pattern()  # [6,4,3]
    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    cells = np.stack([ci, cj, ck], axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)  # cell order i fastest
    corner = cells[:, None, None, :] + pats[None, :, :, :]  # [nc,6,4,3]
    vid = corner[..., 0] + m * (corner[..., 1] + m * corner[..., 2])
    tets = vid.reshape(-1, 4).astype(np.int32)
    return Mesh(xyz=xyz, tets=tets, dirichlet=boundary.astype(np.uint8), n=n, seed=seed)


@dataclass
class KappaField:
    """Parameters of log kappa(x) = sum_k mu_k exp(-|x - c_k|^2 / width).

    kind 'const' means kappa == value everywhere; kind 'per_tet' carries the
    values of every tetrahedron in `value` (one array per mesh level).
    """

    kind: str = "const"
    value: object = 1.0  # float, or per-level arrays for 'per_tet'
    centres: Optional[np.ndarray] = None  # [K,3]
    mu: Optional[np.ndarray] = None  # [K]
    width: float = KAPPA_WIDTH


@dataclass
class LoadField:
    """Values of a source term f on the finest mesh: kind 'per_tet' (one value
    per tetrahedron, f constant on each) or 'nodal' (P1 nodal values)."""

    kind: str
    values: np.ndarray


def kappa_draw(centre_seed: int, mu_seed: int, k: int = 8, mu_range: float = 2.0) -> KappaField:
    """Seeded centres c_k ~ U[0,1]^3 and amplitudes mu ~ U[-2,2]^k."""
    c = np.random.default_rng(centre_seed).uniform(0.0, 1.0, size=(k, 3))
    mu = np.random.default_rng(mu_seed).uniform(-mu_range, mu_range, size=k)
    return KappaField(kind="loggauss", centres=c, mu=mu, width=KAPPA_WIDTH)


def nparts_rule(nv: int) -> int:
    """Subdomain count for a smoothed level without a configured value:
    max(2, 2^floor(log2(nv / 1500)))."""
    q = nv / 1500.0
    if q < 2:
        return 2
    return max(2, 1 << int(np.floor(np.log2(q))))


@dataclass
class Problem:
    """One hierarchy (fine..coarse meshes), its subdomain counts and kappa."""

    name: str
    meshes: List[Mesh]
    nparts: List[int]  # per smoothed level (len L-1); the coarsest is solved directly
    kappa: KappaField
    precision: str = "fp64"  # 'fp64' or 'mixed'
    overlap: int = 1
    its: int = 3
    restart: int = 30
    rtol: float = 1e-8


def coarse_sizes(n: int) -> List[int]:
    """Three-level grid sizes n, n/2, round(n/4.8) (48 -> 24 -> 10)."""
    return [n, n // 2, int(round(n / 4.8))]


def make_hierarchy(ns: Sequence[int], seeds: Sequence[int]) -> List[Mesh]:
    return [kuhn_cube(n, s) for n, s in zip(ns, seeds)]


def cube16_two_level() -> Problem:
    """Plain FP64, two levels: jittered 16^3 fine, independent jittered 6^3
    coarse, kappa = 1, f = 1, 8 subdomains."""
    meshes = make_hierarchy([16, 6], [101, 102])
    return Problem("cube16_6_fp64", meshes, [8], KappaField("const", 1.0))


CUBE48_NPARTS = [64, 32]


def cube48_three_level(precision: str = "fp64") -> Problem:
    """Three levels 48^3 / 24^3 / 10^3, log-Gaussian kappa with 8 seeded
    centres, 64 subdomains on the fine level and 32 on the second (a measured
    choice: the same iteration count as the unknown-count rule's 8 with a
    shorter smoother chain on that level)."""
    meshes = make_hierarchy([48, 24, 10], [201, 202, 203])
    kap = kappa_draw(204, 205)
    name = "cube48_24_10_fp64" if precision == "fp64" else "cube48_24_10_mixed"
    return Problem(name, meshes, list(CUBE48_NPARTS), kap, precision=precision)


def cube32_elasticity(precision: str = "fp64") -> Problem:
    """P1 linear elasticity on jittered 32^3 / 16^3 / 7^3 meshes (seeds
    451-453): Young's modulus from the log-Gaussian field (centres seed 204,
    amplitudes seed 455), three unknowns per vertex, 64 fine-level
    subdomains and the unknown-count rule below; Poisson's ratio and the body
    force are ELASTIC_NU and ELASTIC_FORCE."""
    meshes = make_hierarchy([32, 16, 7], [451, 452, 453])
    return Problem("cube32_elasticity", meshes, [64, nparts_rule(3 * meshes[1].nv)], kappa_draw(204, 455),
                   precision=precision)


ELASTIC_NU = 0.3
ELASTIC_FORCE = (0.0, 0.0, -1.0)


def cube48_three_level_mixed() -> Problem:
    return cube48_three_level("mixed")


def batched_sizes(count: int = 32, seed: int = 400) -> np.ndarray:
    """Fine grid sizes of the batched instances, drawn from {24,32,40,48,64}."""
    return np.random.default_rng(seed).choice(np.array([24, 32, 40, 48, 64]), size=count)


def batched_instances(count: int = 32, precision: str = "mixed") -> List[Problem]:
    """Batched parametric instances with uneven mesh and subdomain sizes."""
    out = []
    sizes = batched_sizes(count)
    for i, n in enumerate(sizes):
        ns = coarse_sizes(int(n))
        meshes = make_hierarchy(ns, [4000 + 10 * i + l for l in range(3)])
        kap = kappa_draw(204, 4000 + 10 * i + 9)
        nps = [nparts_rule(m.nv) for m in meshes[:-1]]
        out.append(Problem(f"batched_{i}_{n}", meshes, nps, kap, precision=precision))
    return out


def served_hierarchy(size: int) -> List[Mesh]:
    """A resident serving hierarchy with fine grid 32, 64 or 96."""
    h = {32: 0, 64: 1, 96: 2}[size]
    return make_hierarchy(coarse_sizes(size), [5000 + 100 * h + l for l in range(3)])


def serving_trace(nreq: int = 2000, rate: float = 10.0, sizes=(32, 64, 96)):
    """Poisson arrivals (exponential gaps, rate per second), hierarchy choice
    uniform, kappa amplitudes per request.  Returns (t_arrival[s], hier_size,
    mu[nreq,8])."""
    gaps = np.random.default_rng(5001).exponential(1.0 / rate, size=nreq)
    t = np.cumsum(gaps)
    hs = np.random.default_rng(5002).choice(np.array(sizes), size=nreq)
    mus = np.stack([np.random.default_rng(5003 + i).uniform(-2.0, 2.0, size=8) for i in range(nreq)])
    return t, hs, mus


def serving_centres() -> np.ndarray:
    return np.random.default_rng(204).uniform(0.0, 1.0, size=(8, 3))


def random_vector(n: int, seed: int, mask: Optional[np.ndarray] = None) -> np.ndarray:
    """A seeded N(0,1) vector, zeroed where mask is nonzero."""
    v = np.random.default_rng(seed).standard_normal(n)
    if mask is not None:
        v[mask.astype(bool)] = 0.0
    return v


def bipyramid_star(hd: float, he: float) -> Mesh:
    """One interior vertex in a triangular bipyramid (a hand-checkable star for
    the coarsening): vertices A, B, C (an equilateral triangle of side 1 in
    z = 0, centroid at the origin, counter-clockwise seen from +z), D =
    (0, 0, hd), E = (0, 0, -he) are Dirichlet; v (id 5) at the origin is the
    only interior vertex.  The six tetrahedra join v to the faces ABD, BCD,
    CAD (above) and BAE, CBE, ACE (below), each positively oriented by the
    counter-clockwise order of A, B, C."""
    r = 1.0 / np.sqrt(3.0)
    xyz = np.array([[r, 0.0, 0.0], [-r / 2, 0.5, 0.0], [-r / 2, -0.5, 0.0],
                    [0.0, 0.0, hd], [0.0, 0.0, -he], [0.0, 0.0, 0.0]])
    A, B, C, D, E, v = range(6)
    tets = np.array([[v, A, B, D], [v, B, C, D], [v, C, A, D],
                     [v, B, A, E], [v, C, B, E], [v, A, C, E]], dtype=np.int32)
    return Mesh(xyz, tets, np.array([1, 1, 1, 1, 1, 0], dtype=np.uint8), 0)

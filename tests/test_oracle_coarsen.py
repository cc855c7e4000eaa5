"""Pins of the oracle's geometry-preserving coarsening (Algorithm 1), no GPU:
the published SplitMix64 sequence, the MIS conditions (1) and (2) of
Section 3.1 and Luby's parallel rounds giving the same set, a hand-checked
single vertex removal, and mesh invariants of the output (positive volumes,
the unit volume, conformity, the boundary surface kept triangle by triangle,
Euler characteristic of a ball)."""
import os
from collections import Counter

import numpy as np
import pytest

import workloads as W
from oracle import coarsen, problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def test_splitmix64_published_sequence():
    ref = [int(l, 16) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    gold = 0x9E3779B97F4A7C15
    got = [coarsen.splitmix64((k * gold) & coarsen.MASK) for k in range(3)]
    assert got == ref


def _faces(tets):
    c = Counter()
    for t in tets:
        for f in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
            c[tuple(sorted(int(t[i]) for i in f))] += 1
    return c


@pytest.mark.parametrize("seed,rnd", [(7, 0), (11, 3)])
def test_mis_conditions_and_luby_rounds(seed, rnd):
    m = W.kuhn_cube(7, 3)
    T = [list(t) for t in m.tets]
    alive = [True] * m.nv
    bnd = [bool(d) for d in m.dirichlet]
    S, nb = coarsen.mis(m.nv, T, alive, bnd, seed, rnd)
    Sset = set(S)
    cand = [v for v in range(m.nv) if not bnd[v]]
    # (1) independence, (2) maximality among the interior vertices
    for v in S:
        assert not (nb[v] & Sset)
    for v in cand:
        assert v in Sset or (nb[v] & Sset)
    # Luby's parallel rounds with the same priorities: a vertex joins when
    # its key is below every undecided neighbour's; it and its neighbours
    # leave; repeat
    key = {v: (coarsen.priority(seed, rnd, v), v) for v in cand}
    und = set(cand)
    L = set()
    while und:
        joins = {v for v in und if all(key[v] < key[w] for w in nb[v] if w in und)}
        L |= joins
        und -= joins
        und -= {w for v in joins for w in nb[v]}
    assert L == Sset


def test_single_cavity_by_hand():
    # unit cube split into 12 tetrahedra coned from its centre: the only
    # interior vertex is removed and the cavity becomes the cone from the
    # chosen corner over the three cube faces that do not contain it
    corners = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=float)
    xyz = np.vstack([corners, [[0.5, 0.5, 0.5]]])
    quads = [(0, 1, 3, 2), (4, 5, 7, 6), (0, 1, 5, 4), (2, 3, 7, 6), (0, 2, 6, 4), (1, 3, 7, 5)]
    tets = []
    for a, b, c, d in quads:
        for tri in ((a, b, c), (a, c, d)):
            t = [tri[0], tri[1], tri[2], 8]
            if coarsen.det6(*(xyz[i] for i in t)) < 0:
                t[0], t[1] = t[1], t[0]
            tets.append(t)
    dmask = np.array([1] * 8 + [0], dtype=np.uint8)
    r = coarsen.coarsen(xyz, np.array(tets), dmask, 1, 5)
    assert r.removed == 1 and len(r.xyz) == 8 and len(r.tets) == 6
    vols = [coarsen.det6(*(r.xyz[i] for i in t)) / 6 for t in r.tets]
    assert min(vols) > 0 and abs(sum(vols) - 1.0) <= 1e-15
    # the new elements are the cones from one corner u over the surface
    # triangles that do not contain u
    surf = {tuple(sorted(tri)) for a, b, c, d in quads for tri in ((a, b, c), (a, c, d))}
    common = set(r.tets[0])
    for t in r.tets:
        common &= set(int(x) for x in t)
    old = {i: int(o) for i, o in enumerate(r.kept_ids)}
    ok = False
    for u in common:
        cones = {tuple(sorted(old[int(x)] for x in t if x != u)) for t in r.tets}
        ok |= cones == {f for f in surf if old[u] not in f}
    assert ok


@pytest.mark.parametrize("n,rounds,seed", [(7, 1, 3), (9, 8, 7), (12, 4, 19)])
def test_output_mesh_invariants(n, rounds, seed):
    m = W.kuhn_cube(n, seed)
    r = coarsen.coarsen(m.xyz, m.tets, m.dirichlet, rounds, seed)
    assert r.removed > 0 and len(r.xyz) == m.nv - r.removed
    vols = np.array([coarsen.det6(*(r.xyz[i] for i in t)) for t in r.tets]) / 6
    assert vols.min() > 0
    assert abs(vols.sum() - 1.0) <= 1e-12
    F = _faces(r.tets)
    assert max(F.values()) <= 2
    # boundary surface kept triangle by triangle (through the kept ids)
    Ff = _faces(m.tets)
    bf = {f for f, c in Ff.items() if c == 1}
    kept = {int(o): i for i, o in enumerate(r.kept_ids)}
    bc = {f for f, c in F.items() if c == 1}
    assert bc == {tuple(sorted(kept[a] for a in f)) for f in bf}
    # only interior vertices go; every vertex is used; Euler characteristic
    assert np.all(m.dirichlet[r.kept_ids] == r.dirichlet)
    assert int(m.dirichlet.sum()) == int(r.dirichlet.sum())
    assert len(np.unique(r.tets)) == len(r.xyz)
    E = set()
    for t in r.tets:
        for i in range(4):
            for j in range(i + 1, 4):
                E.add((min(t[i], t[j]), max(t[i], t[j])))
    assert len(r.xyz) - len(E) + len(F) - len(r.tets) == 1
    # the new elements respect the quality floor
    q = [coarsen.quality(*(r.xyz[i] for i in t)) for t in r.tets]
    assert min(q) > 0


def test_zero_rounds_is_identity():
    m = W.kuhn_cube(5, 2)
    r = coarsen.coarsen(m.xyz, m.tets, m.dirichlet, 0, 1)
    assert r.removed == 0 and np.array_equal(r.tets, m.tets) and np.array_equal(r.xyz, m.xyz)


def test_coarsened_hierarchy_converges():
    m = W.kuhn_cube(12, 5)
    r = coarsen.coarsen(m.xyz, m.tets, m.dirichlet, 8, 5)
    c = W.Mesh(r.xyz, r.tets.astype(np.int32), r.dirichlet, 0)
    pb = W.Problem("coarsened", [m, c], [4], W.kappa_draw(204, 205))
    h = problem.build(pb)
    res = problem.solve(h)
    assert res.converged
    x = problem.exact(h)
    assert np.linalg.norm(res.x - x) <= 1e-6 * np.linalg.norm(x)


QGOLD = os.path.join(os.path.dirname(__file__), "golden", "tet_quality.txt")


def quality_golden():
    """Rows of tests/golden/tet_quality.txt: {name: (hd, he, q_abc_min,
    q_abc_mean, q_de, expected)} and the Kuhn tetrahedron's quality."""
    rows, kuhn = {}, None
    for line in open(QGOLD):
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "kuhn_q":
            kuhn = float(f[1])
        else:
            rows[f[0]] = tuple(float(x) for x in f[1:6]) + (f[6],)
    return rows, kuhn


def expected_star_tets(kind):
    """Vertex sets of the elements a bipyramid star leaves (ids A..E = 0..4)."""
    A, B, C, D, E = range(5)
    if kind == "abc":
        return {frozenset((A, B, C, D)), frozenset((A, B, C, E))}
    return {frozenset((D, E, A, B)), frozenset((D, E, B, C)), frozenset((D, E, C, A))}


def test_quality_closed_forms():
    """q = 1 for a regular tetrahedron whatever its position, size and
    rotation (and -1 mirrored), sqrt(2) (3/5)^(3/2) for the Kuhn
    tetrahedron, 0 for a flat one: fixes the constant, the volume and that
    l_rms is the root mean square of the edges (a mean edge gives 0.7068 on
    the Kuhn tetrahedron)."""
    _, kuhn = quality_golden()
    reg = np.array([[1, -1, -1], [1, 1, 1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
    assert coarsen.det6(*reg) > 0
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    for scale, shift in ((1.0, 0.0), (0.37, 5.0), (12.5, -3.25)):
        p = reg @ Q.T * scale + shift
        assert abs(coarsen.quality(*p) - 1.0) <= 1e-14
        assert abs(coarsen.quality(p[1], p[0], p[2], p[3]) + 1.0) <= 1e-14
    k = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1]], dtype=float)
    assert abs(coarsen.quality(*k) - kuhn) <= 1e-15
    assert abs(coarsen.quality(*(0.01 * k + 0.5)) - kuhn) <= 1e-13
    flat = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.3, 0.4, 0]], dtype=float)
    assert coarsen.quality(*flat) == 0.0


@pytest.mark.parametrize("name", ["regular", "lopsided", "flat02", "flat007", "flat005"])
def test_contraction_choice_on_hand_checked_stars(name):
    """The removed vertex goes to the neighbour whose new elements have the
    largest smallest quality, and only above the floor 0.02 (Section 3.1,
    reading of the cavity re-meshing): the bipyramid stars of the golden
    file, whose qualities are closed forms, leave the elements fixed by hand
    ('lopsided' needs the smallest quality: the mean or the largest would
    take A, B or C)."""
    rows, _ = quality_golden()
    hd, he, q_abc_min, q_abc_mean, q_de, expected = rows[name]
    m = W.bipyramid_star(hd, he)
    r = coarsen.coarsen(m.xyz, m.tets, m.dirichlet, 1, 9)
    if expected == "keep":
        assert r.removed == 0 and np.array_equal(r.tets, m.tets)
        assert max(q_abc_min, q_de) < coarsen.QMIN
        return
    assert r.removed == 1 and list(r.kept_ids) == [0, 1, 2, 3, 4]
    got = {frozenset(int(x) for x in t) for t in r.tets}
    assert got == expected_star_tets(expected)
    q = [coarsen.quality(*(r.xyz[i] for i in t)) for t in r.tets]
    assert min(q) > 0
    assert abs(min(q) - (q_abc_min if expected == "abc" else q_de)) <= 1e-13

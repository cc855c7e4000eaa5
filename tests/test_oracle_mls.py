"""Pins of the oracle's moving-least-squares interpolation (Section 3.2), no
GPU.  Each check comes from something other than the oracle's own formula:
a factored closed form of the weight, a library weighted least-squares
solve, barycentric coordinates as volume ratios, exact reproduction of
linear functions, and Theorem 1's rank condition."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import workloads as W
from oracle import mls, problem


def test_weight_closed_form_and_support():
    r = np.linspace(0.0, 1.0, 1001)
    # the quartic factors as (1 - r)^3 (1 + 3 r): positive on [0, 1), a
    # triple root at r = 1 (w, w' and w'' vanish at the support's edge)
    np.testing.assert_allclose(mls.weight(r), (1 - r) ** 3 * (1 + 3 * r), atol=1e-15)
    assert mls.weight(0.0) == 1.0
    assert abs(mls.weight(1.0)) < 1e-15
    assert np.all(mls.weight(r[:-1]) > 0)
    eps = 1e-5
    assert abs((mls.weight(1.0) - mls.weight(1.0 - eps)) / eps) < 1e-8
    assert np.all(np.diff(mls.weight(r)) < 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_row_is_the_weighted_least_squares_fit(seed):
    rng = np.random.default_rng(seed)
    xs = rng.uniform(-1, 1, 3)
    pts = xs + rng.uniform(-0.3, 0.3, (17, 3))
    rho = 1.05 * np.linalg.norm(pts - xs, axis=1).max()
    u = rng.standard_normal(len(pts))
    w = mls.weight(np.linalg.norm(pts - xs, axis=1) / rho)
    # argmin sum w (a0 + a.x - u)^2 by a library least-squares solve
    M = np.hstack([np.ones((len(pts), 1)), pts]) * np.sqrt(w)[:, None]
    a, *_ = np.linalg.lstsq(M, np.sqrt(w) * u, rcond=None)
    ref = a[0] + a[1:] @ xs
    assert abs(mls.mls_row(xs, pts, rho) @ u - ref) <= 1e-12 * (1 + abs(ref))


def _vol(a, b, c, d):
    return np.linalg.det(np.array([b - a, c - a, d - a])) / 6.0


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_four_neighbours_give_barycentric_coordinates(seed):
    rng = np.random.default_rng(seed)
    T = rng.uniform(0, 1, (4, 3))
    lam = rng.dirichlet(np.ones(4))
    xs = lam @ T
    rho = 1.01 * np.linalg.norm(T - xs, axis=1).max()
    phi = mls.mls_row(xs, T, rho)
    # barycentric coordinates as ratios of signed volumes
    V = _vol(*T)
    ref = []
    for i in range(4):
        Ti = T.copy()
        Ti[i] = xs
        ref.append(_vol(*Ti) / V)
    np.testing.assert_allclose(phi, ref, atol=1e-12)
    np.testing.assert_allclose(phi, lam, atol=1e-12)


@pytest.mark.parametrize("nf,nc,sf,sc,alpha", [(6, 3, 1, 2, 1.5), (9, 4, 3, 4, 1.0), (9, 5, 7, 8, 2.0)])
def test_reproduces_linear_functions(nf, nc, sf, sc, alpha):
    f, c = W.kuhn_cube(nf, sf), W.kuhn_cube(nc, sc)
    P = mls.interpolation(f, c, alpha, mask_dirichlet=False)
    for coef in ([0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0.7, -1.3, 2.1, 0.4]):
        gc = c.xyz @ np.array(coef[:3]) + coef[3]
        gf = f.xyz @ np.array(coef[:3]) + coef[3]
        assert np.abs(P @ gc - gf).max() <= 1e-12
    rs = np.asarray(P.sum(axis=1)).ravel()
    assert np.abs(rs - 1).max() <= 1e-12
    # a quadratic is not reproduced: the operator is not the identity on it
    q = lambda x: (x ** 2).sum(axis=1)
    assert np.abs(P @ q(c.xyz) - q(f.xyz)).max() > 1e-4


def test_neighbourhood_matches_brute_force():
    c = W.kuhn_cube(7, 11)
    f = W.kuhn_cube(11, 12)
    h = mls.mean_edge_length(c.xyz, c.tets)
    tree = cKDTree(c.xyz)
    for v in range(0, f.nv, 37):
        ids, rho = mls.neighbourhood(tree, c.xyz, f.xyz[v], 1.5 * h)
        d = np.linalg.norm(c.xyz - f.xyz[v], axis=1)
        assert np.array_equal(ids, np.nonzero(d < rho)[0])


def test_mean_edge_length_by_brute_force():
    m = W.kuhn_cube(4, 5)
    E = set()
    for t in m.tets:
        for i in range(4):
            for j in range(i + 1, 4):
                E.add((min(t[i], t[j]), max(t[i], t[j])))
    ref = np.mean([np.linalg.norm(m.xyz[a] - m.xyz[b]) for a, b in E])
    assert abs(mls.mean_edge_length(m.xyz, m.tets) - ref) <= 1e-14


def test_rank_deficient_neighbourhood_grows_rho():
    # Theorem 1: coplanar neighbours leave rank(P) = 3 < 4; the scale must
    # grow until the off-plane node at distance 1.0 is strictly inside
    g = np.linspace(-0.3, 0.3, 7)
    plane = np.array([(x, y, 0.0) for x in g for y in g])
    src = np.vstack([plane, [[0.0, 0.0, 1.0]]])
    xs = np.array([0.01, 0.02, 0.1])
    assert not mls.full_rank(xs, plane, 0.5)
    ids, rho = mls.neighbourhood(cKDTree(src), src, xs, 0.5)
    assert rho > np.linalg.norm(src[-1] - xs)
    assert len(src) - 1 in ids
    assert mls.full_rank(xs, src[ids], rho)
    phi = mls.mls_row(xs, src[ids], rho)
    for coef in ([1, 0, 0, 0], [0, 0, 1, 0], [0.3, -0.2, 1.7, 0.5]):
        val = src[ids] @ np.array(coef[:3]) + coef[3]
        assert abs(phi @ val - (xs @ np.array(coef[:3]) + coef[3])) <= 1e-12


def test_too_few_points_are_not_full_rank():
    xs = np.zeros(3)
    pts = np.eye(3) * 0.1
    assert not mls.full_rank(xs, pts, 1.0)


def test_dirichlet_masking():
    f, c = W.kuhn_cube(7, 1), W.kuhn_cube(4, 2)
    P = mls.interpolation(f, c, 1.5).tocsr()
    Pu = mls.interpolation(f, c, 1.5, mask_dirichlet=False).tocsr()
    for v in range(f.nv):
        cols = P.indices[P.indptr[v]:P.indptr[v + 1]]
        if f.dirichlet[v]:
            assert len(cols) == 0
            continue
        assert np.all(c.dirichlet[cols] == 0)
        # the masked row is the unmasked one without its Dirichlet columns
        cu = Pu.indices[Pu.indptr[v]:Pu.indptr[v + 1]]
        vu = Pu.data[Pu.indptr[v]:Pu.indptr[v + 1]]
        keep = c.dirichlet[cu] == 0
        row = dict(zip(cols, P.data[P.indptr[v]:P.indptr[v + 1]]))
        assert set(row) == set(cu[keep])
        for k, val in zip(cu[keep], vu[keep]):
            assert row[k] == val


def test_vcycle_with_mls_transfer_converges():
    pb = W.cube16_two_level()
    h = problem.build(pb, mls_alpha=1.5)
    r = problem.solve(h)
    assert r.converged
    x = problem.exact(h)
    assert np.linalg.norm(r.x - x) <= 1e-6 * np.linalg.norm(x)


def test_clipped_neighbourhoods():
    """The paper's neighbourhood clipped to the overlapping subdomain of the
    target's processor (Section 3.2): every row's support lies in that
    subdomain's nodes, linear functions are still reproduced exactly, and a
    row whose unclipped neighbourhood already lies inside the subdomain is
    the same row."""
    fine, coarse = W.kuhn_cube(9, 71), W.kuhn_cube(5, 72)
    owner, masks = mls.clip_sets(fine, coarse, 4, 1)
    Pc = mls.interpolation(fine, coarse, mls.ALPHA, mask_dirichlet=False, clip=(owner, masks)).tocsr()
    Pu = mls.interpolation(fine, coarse, mls.ALPHA, mask_dirichlet=False).tocsr()
    lin = lambda X: 0.3 + 1.1 * X[:, 0] - 0.7 * X[:, 1] + 2.0 * X[:, 2]
    inner = fine.dirichlet == 0
    assert np.abs((Pc @ lin(coarse.xyz) - lin(fine.xyz))[inner]).max() <= 1e-12
    same = 0
    for v in np.nonzero(inner)[0]:
        cols = Pc.indices[Pc.indptr[v]:Pc.indptr[v + 1]]
        assert masks[owner[v]][cols].all(), v
        ucols = Pu.indices[Pu.indptr[v]:Pu.indptr[v + 1]]
        if masks[owner[v]][ucols].all():
            same += 1
            assert np.array_equal(np.sort(cols), np.sort(ucols))
            assert np.abs(Pc[v].toarray() - Pu[v].toarray()).max() <= 1e-14
    assert same > 0.5 * inner.sum()
    # some interior rows do change: the clipping is not vacuous
    assert abs(Pc[np.nonzero(inner)[0]] - Pu[np.nonzero(inner)[0]]).max() > 1e-6


def test_clipped_vcycle_converges():
    pb = W.Problem("clip", [W.kuhn_cube(10, 73), W.kuhn_cube(6, 74), W.kuhn_cube(3, 75)], [4, 2],
                   W.kappa_draw(204, 205))
    h = problem.build(pb, mls_alpha=1.0, mls_clip=True)
    res = problem.solve(h)
    xs = problem.exact(h)
    assert res.converged and np.linalg.norm(res.x - xs) <= 1e-7 * np.linalg.norm(xs)

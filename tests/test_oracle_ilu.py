"""Pins of the oracle's ILU(k) subdomain solver (no GPU): the fill-path
characterisation of the level of fill checked by brute force, the defining
property of an incomplete factorisation (L U = A on the pattern), exact LU
when nothing is dropped, and textbook fill patterns."""
from collections import deque

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import ilu, problem, schwarz


def _random_spd(n, density, seed):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, data_rvs=lambda k: -rng.uniform(0.1, 1.0, k))
    M = sp.triu(M, 1)
    M = M + M.T
    d = np.asarray(abs(M).sum(axis=1)).ravel() + rng.uniform(0.5, 1.5, n)
    return (M + sp.diags(d)).tocsr()


def _fill_levels_by_paths(A, k):
    """Entry (i, j) has level m-1 where m is the length of the shortest path
    i -> j in the graph of A whose inner vertices are all below min(i, j)
    (the fill-path theorem); kept when that level is <= k."""
    n = A.shape[0]
    adj = [set(A.indices[A.indptr[i]:A.indptr[i + 1]]) - {i} for i in range(n)]
    out = {}
    for i in range(n):
        for j in range(n):
            if i == j:
                out[(i, j)] = 0
                continue
            lim = min(i, j)
            dist = {i: 0}
            q = deque([i])
            found = None
            while q and found is None:
                v = q.popleft()
                for w in adj[v]:
                    if w == j:
                        found = dist[v] + 1
                        break
                    if w < lim and w not in dist:
                        dist[w] = dist[v] + 1
                        q.append(w)
            if found is not None and found - 1 <= k:
                out[(i, j)] = found - 1
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("fill", [0, 1, 2, 3])
def test_pattern_is_the_fill_path_set(seed, fill):
    A = _random_spd(16, 0.15, seed)
    cols, levs = ilu.symbolic(A, fill)
    got = {(i, int(j)): int(l) for i in range(16) for j, l in zip(cols[i], levs[i])}
    assert got == _fill_levels_by_paths(A, fill)


@pytest.mark.parametrize("fill", [0, 1, 2])
def test_lu_equals_a_on_the_pattern(fill):
    A = _random_spd(40, 0.08, 7)
    cols, _ = ilu.symbolic(A, fill)
    L, U = ilu.factor(A, cols)
    LU = (L @ U).toarray()
    Ad = A.toarray()
    for i in range(40):
        for j in cols[i]:
            assert abs(LU[i, j] - Ad[i, j]) <= 1e-12 * abs(Ad).max()
    # the patterns of L and U are exactly the symbolic one
    assert set(zip(*sp.triu(U).nonzero())) | set(zip(*sp.tril(L, -1).nonzero())) <= \
        {(i, int(j)) for i in range(40) for j in cols[i]}


def test_no_dropping_gives_the_exact_factorisation():
    A = _random_spd(30, 0.1, 9)
    f = ilu.ILU(A, 30)
    np.testing.assert_allclose((f.L @ f.U).toarray(), A.toarray(), atol=1e-12)
    r = np.random.default_rng(0).standard_normal(30)
    np.testing.assert_allclose(f.solve(r), np.linalg.solve(A.toarray(), r), rtol=1e-10)


def test_tridiagonal_ilu0_is_exact():
    n = 25
    A = sp.diags([-np.ones(n - 1), 2.5 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    f = ilu.ILU(A, 0)
    r = np.arange(n, dtype=float)
    np.testing.assert_allclose(f.solve(r), np.linalg.solve(A.toarray(), r), rtol=1e-12)


def test_five_point_grid_fill_positions():
    # lexicographic 5-point Laplacian: ILU(0) keeps the pattern, ILU(1)
    # adds exactly the entries at offsets +-(nx - 1) inside the grid
    nx = 6
    T = sp.diags([-np.ones(nx - 1), 4 * np.ones(nx), -np.ones(nx - 1)], [-1, 0, 1])
    A = (sp.kron(sp.identity(nx), T) + sp.kron(sp.diags([-np.ones(nx - 1), -np.ones(nx - 1)], [-1, 1]),
                                                 sp.identity(nx))).tocsr()
    A.sort_indices()
    c0, _ = ilu.symbolic(A, 0)
    for i in range(nx * nx):
        assert np.array_equal(c0[i], A.indices[A.indptr[i]:A.indptr[i + 1]])
    c1, l1 = ilu.symbolic(A, 1)
    for i in range(nx * nx):
        extra = sorted(set(c1[i]) - set(A.indices[A.indptr[i]:A.indptr[i + 1]]))
        expect = [j for j in (i - nx + 1, i + nx - 1) if 0 <= j < nx * nx
                  and ((j == i + nx - 1 and i % nx != 0) or (j == i - nx + 1 and i % nx != nx - 1))]
        assert extra == expect, (i, extra, expect)
        assert all(l == 1 for j, l in zip(c1[i], l1[i]) if j in extra)


def test_nonpositive_pivot_is_an_error():
    A = sp.csr_matrix(np.array([[1.0, 2.0], [2.0, 1.0]]))
    with pytest.raises(ZeroDivisionError):
        ilu.ILU(A, 0)


def test_ras_with_full_fill_one_subdomain_is_exact():
    pb = W.Problem("one", [W.kuhn_cube(5, 41), W.kuhn_cube(3, 42)], [1], W.kappa_draw(1, 2), overlap=0)
    h = problem.build(pb)
    A = h.A[0]
    owned, sets = schwarz.partition(pb.meshes[0], 1, 0)
    ras = schwarz.RAS(A, pb.meshes[0].dirichlet, owned, sets, ilu_fill=A.shape[0])
    r = np.random.default_rng(3).standard_normal(A.shape[0])
    r[pb.meshes[0].dirichlet != 0] = 0
    z = ras.apply(r)
    assert np.linalg.norm(A @ z - r) <= 1e-10 * np.linalg.norm(r)


@pytest.mark.parametrize("fill", [[0], [2]])
def test_vcycle_with_ilu_converges(fill):
    pb = W.cube16_two_level()
    h = problem.build(pb, ilu_fill=fill)
    r = problem.solve(h)
    assert r.converged
    x = problem.exact(h)
    assert np.linalg.norm(r.x - x) <= 1e-6 * np.linalg.norm(x)

"""Pins of the oracle's partition, overlap, RAS, V-cycle and FGMRES (no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import fem, krylov, multilevel, problem, schwarz, transfer


def _system(n, seed, kappa=None):
    m = W.kuhn_cube(n, seed)
    A, b = fem.assemble(m, kappa or W.KappaField(), 1.0)
    return m, A, b


def _ring_from_tets(m, own):
    """Independent 1-ring: every interior vertex of a tetrahedron that has a
    vertex in own."""
    ownset = np.zeros(m.nv, dtype=bool)
    ownset[own] = True
    hit = ownset[m.tets].any(axis=1)
    ring = np.unique(m.tets[hit].ravel())
    return np.sort(ring[m.dirichlet[ring] == 0])


@pytest.mark.parametrize("nparts", [1, 2, 8])
def test_partition_owned_sets_and_overlap(nparts):
    m = W.kuhn_cube(8, 31)
    owned, sets = schwarz.partition(m, nparts, overlap=1)
    interior = np.nonzero(m.dirichlet == 0)[0]
    allown = np.sort(np.concatenate(owned))
    assert np.array_equal(allown, interior)  # a partition: disjoint, covering
    sizes = [len(o) for o in owned]
    assert max(sizes) - min(sizes) <= 1
    for own, S in zip(owned, sets):
        assert np.all(np.diff(S) > 0)
        assert np.array_equal(S, _ring_from_tets(m, own))
    owned0, sets0 = schwarz.partition(m, nparts, overlap=0)
    for own, S in zip(owned0, sets0):
        assert np.array_equal(np.sort(own), S)


def test_rcb_splits_along_axes():
    m = W.kuhn_cube(8)  # un-jittered: the first cut is the plane x = 1/2
    owned, _ = schwarz.partition(m, 2, overlap=0)
    x0 = m.xyz[owned[0], 0]
    x1 = m.xyz[owned[1], 0]
    assert x0.max() <= x1.min()
    owned4, _ = schwarz.partition(m, 4, overlap=0)
    # second cut along y inside each half
    assert m.xyz[owned4[0], 1].max() <= m.xyz[owned4[1], 1].min()
    assert m.xyz[owned4[0], 0].max() <= m.xyz[owned4[2], 0].min()


def test_one_subdomain_no_overlap_is_exact():
    m, A, b = _system(6, 41, W.kappa_draw(1, 2))
    owned, sets = schwarz.partition(m, 1, overlap=0)
    ras = schwarz.RAS(A, m.dirichlet, owned, sets)
    B = ras.dense(m.nv)
    assert np.abs(B @ A.toarray() - np.eye(m.nv)).max() <= 1e-10
    res = krylov.fgmres(A, b, ras.apply, restart=30, rtol=1e-8)
    assert res.iterations == 1 and res.relres <= 1e-13


def test_full_overlap_is_exact():
    """With so much overlap that every S_p is the whole interior, every
    subdomain solves exactly and RAS keeps the owned parts: B = A^{-1}.
    This pins the restriction (R^0)^T, i.e. the owned positions."""
    m, A, _ = _system(4, 42)
    owned, sets = schwarz.partition(m, 4, overlap=10)
    assert all(len(S) == int((m.dirichlet == 0).sum()) for S in sets)
    B = schwarz.RAS(A, m.dirichlet, owned, sets).dense(m.nv)
    assert np.abs(B @ A.toarray() - np.eye(m.nv)).max() <= 1e-10


def test_no_overlap_is_block_jacobi():
    m, A, _ = _system(5, 43, W.kappa_draw(3, 4))
    owned, sets = schwarz.partition(m, 4, overlap=0)
    B = schwarz.RAS(A, m.dirichlet, owned, sets).dense(m.nv)
    BA = B @ A.toarray()
    for own in owned:
        blk = BA[np.ix_(own, own)]
        assert np.abs(blk - np.eye(len(own))).max() <= 1e-10


def test_ras_restricts_to_owned_rows():
    """RAS with overlap differs from plain additive Schwarz: summing over
    subdomains the extended (not restricted) solutions gives another
    operator.  Pins that only owned rows are written."""
    m, A, _ = _system(5, 44)
    owned, sets = schwarz.partition(m, 2, overlap=1)
    ras = schwarz.RAS(A, m.dirichlet, owned, sets)
    r = np.random.default_rng(0).standard_normal(m.nv)
    r[m.dirichlet != 0] = 0
    z = ras.apply(r)
    Ad = A.toarray()
    for own, S in zip(owned, sets):
        y = np.linalg.solve(Ad[np.ix_(S, S)], r[S])
        pos = np.searchsorted(S, own)
        np.testing.assert_allclose(z[own], y[pos], rtol=1e-12, atol=1e-14)


def _two_level(nf, nc, nparts, sf=5, sc=6, overlap=1, its=3):
    f, c = W.kuhn_cube(nf, sf), W.kuhn_cube(nc, sc)
    Af, bf = fem.assemble(f, W.KappaField(), 1.0)
    Ac, _ = fem.assemble(c, W.KappaField(), 1.0)
    P = transfer.interpolation(f, c)
    owned, sets = schwarz.partition(f, nparts, overlap)
    ras = schwarz.RAS(Af, f.dirichlet, owned, sets)
    levels = [multilevel.Level(Af, f.dirichlet, ras, P), multilevel.Level(Ac, c.dirichlet)]
    return f, c, Af, Ac, bf, P, ras, multilevel.VCycle(levels, its)


def test_vcycle_with_identical_coarse_mesh_is_exact():
    f = W.kuhn_cube(5, 7)
    A, b = fem.assemble(f, W.KappaField(), 1.0)
    P = transfer.interpolation(f, f)
    owned, sets = schwarz.partition(f, 4, 1)
    ras = schwarz.RAS(A, f.dirichlet, owned, sets)
    vc = multilevel.VCycle([multilevel.Level(A, f.dirichlet, ras, P), multilevel.Level(A, f.dirichlet)], 3)
    M = np.stack([vc(e) for e in np.eye(f.nv)], axis=1)
    assert np.abs(M @ A.toarray() - np.eye(f.nv)).max() <= 1e-10


def test_two_level_error_propagation_identity():
    """I - M A = E^its (I - P A_c^{-1} P^T A) E^its with E = I - B A: the
    error propagation of Algorithm 2 written as a product of operators."""
    f, c, Af, Ac, _, P, ras, vc = _two_level(5, 3, 4)
    n = f.nv
    Ad = Af.toarray()
    B = ras.dense(n)
    E = np.eye(n) - B @ Ad
    Pd = P.toarray()
    C = np.eye(n) - Pd @ np.linalg.solve(Ac.toarray(), Pd.T @ Ad)
    E3 = np.linalg.matrix_power(E, 3)
    expected = E3 @ C @ E3
    M = np.stack([vc(e) for e in np.eye(n)], axis=1)
    assert np.abs((np.eye(n) - M @ Ad) - expected).max() <= 1e-10
    # a mistake in the step order (e.g. a missing post-smoothing) would not match
    assert np.abs(E3 @ C - expected).max() > 1e-6


def test_fgmres_arnoldi_relation_and_true_residual():
    f, c, Af, Ac, bf, P, ras, vc = _two_level(6, 3, 4, its=1)
    res = krylov.fgmres(Af, bf, lambda v: v + 0.0 * v, restart=10, rtol=1e-30, max_it=10)
    k = 10
    V, Z, H = res.V, res.Z, res.H
    assert np.abs(Af @ Z[:, :k] - V[:, : k + 1] @ H[: k + 1, :k]).max() <= 1e-12 * np.abs(Af.data).max()
    assert np.abs(V[:, : k + 1].T @ V[:, : k + 1] - np.eye(k + 1)).max() <= 1e-12
    # the Givens estimate equals the true residual of x
    true = np.linalg.norm(bf - Af @ res.x) / np.linalg.norm(bf)
    assert abs(res.history[-1] - true) <= 1e-10 * max(true, 1e-300) + 1e-15


@pytest.mark.parametrize("nf", [2, 3, 4])
def test_bruteforce_tiny_solves_agree(nf):
    """Dense numpy solve == sparse direct x* == the FGMRES + V-cycle result."""
    nc = max(1, nf - 1)
    pb = W.Problem("tiny", [W.kuhn_cube(nf, 60 + nf), W.kuhn_cube(nc, 70 + nf)], [2], W.kappa_draw(5, 6))
    h = problem.build(pb, locate=transfer.locate_bruteforce)
    xd = np.linalg.solve(h.A[0].toarray(), h.b)
    xs = problem.exact(h)
    res = problem.solve(h)
    assert res.converged and res.relres <= 1e-8
    np.testing.assert_allclose(xs, xd, rtol=1e-12, atol=1e-15)
    assert np.linalg.norm(res.x - xd) <= 1e-7 * np.linalg.norm(xd)


def test_multilevel_beats_one_level():
    """Soft trend of the paper's tables: more levels, fewer iterations."""
    f = W.kuhn_cube(12, 81)
    A, b = fem.assemble(f, W.KappaField(), 1.0)
    owned, sets = schwarz.partition(f, 8, 1)
    ras = schwarz.RAS(A, f.dirichlet, owned, sets)
    one = krylov.fgmres(A, b, ras.apply, 30, 1e-8)
    c = W.kuhn_cube(5, 82)
    Ac, _ = fem.assemble(c, W.KappaField(), 1.0)
    vc = multilevel.VCycle([multilevel.Level(A, f.dirichlet, ras, transfer.interpolation(f, c)),
                            multilevel.Level(Ac, c.dirichlet)], 3)
    two = krylov.fgmres(A, b, vc, 30, 1e-8)
    assert two.converged and one.converged
    assert two.iterations < one.iterations

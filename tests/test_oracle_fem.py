"""Pins of the oracle's P1 discretisation against closed forms, invariants and
a convergence rate (no GPU)."""
import os
from math import factorial

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import fem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLD, name), comments="#")


def test_mesh_volumes_tile_the_cube():
    for n, s in [(1, None), (3, 7), (16, 101), (24, 202)]:
        m = W.kuhn_cube(n, s)
        vol = fem.check_mesh(m.xyz, m.tets)
        assert np.all(vol > 0)
        assert abs(vol.sum() - 1.0) <= 1e-14 * max(1, m.nt) ** 0.5 * 10
        assert m.nv == (n + 1) ** 3 and m.nt == 6 * n ** 3


def test_reference_tet_stiffness_golden():
    K = _load("p1_reference_tet_stiffness.txt") / 6.0
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
    tets = np.array([[0, 1, 2, 3]], dtype=np.int32)
    A = fem.stiffness_neumann(xyz, tets, W.KappaField()).toarray()
    np.testing.assert_allclose(A, K, atol=1e-15)
    # kappa scales linearly; an affine map x -> 2x scales the stiffness by 2
    A2 = fem.stiffness_neumann(2 * xyz, tets, W.KappaField("const", 3.0)).toarray()
    np.testing.assert_allclose(A2, 6 * K, atol=1e-14)


def test_kuhn_stencil_golden():
    st = _load("kuhn_p1_stencil.txt")
    n = 4
    h = 1.0 / n
    m = W.kuhn_cube(n)
    A = fem.stiffness_neumann(m.xyz, m.tets, W.KappaField()).tocsr()
    for (ci, cj, ck) in [(1, 1, 1), (2, 2, 2), (1, 2, 3)]:
        i = ci + 5 * (cj + 5 * ck)
        row = A[i].toarray().ravel()
        seen = set()
        for di, dj, dk, val in st:
            j = (ci + int(di)) + 5 * ((cj + int(dj)) + 5 * (ck + int(dk)))
            assert abs(row[j] - val * h) <= 1e-14, (di, dj, dk)
            seen.add(j)
        # the pattern of the mesh graph is exactly these 15 entries
        assert set(A[i].indices) == seen


@pytest.mark.parametrize("seed", [11, 12])
def test_stiffness_symmetric_rowsum_zero_any_kappa(seed):
    m = W.kuhn_cube(6, seed)
    kap = W.kappa_draw(seed, seed + 1)
    A = fem.stiffness_neumann(m.xyz, m.tets, kap)
    amax = np.abs(A.data).max()
    assert abs(A - A.T).max() <= 1e-15 * amax
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert np.abs(rs).max() <= 1e-13 * amax
    # positive diagonal, SPD after elimination
    Ad, _ = fem.dirichlet_eliminate(A, np.zeros(m.nv), m.dirichlet)
    ev = np.linalg.eigvalsh(Ad.toarray())
    assert ev.min() > 0


def test_patch_test_linear_functions():
    m = W.kuhn_cube(5, 3)
    A = fem.stiffness_neumann(m.xyz, m.tets, W.KappaField("const", 2.5))
    interior = m.dirichlet == 0
    for c in ([1, 0, 0, 0], [0, 1, 0, 0], [0.3, -2, 1.5, 0.7]):
        ell = c[0] * m.xyz[:, 0] + c[1] * m.xyz[:, 1] + c[2] * m.xyz[:, 2] + c[3]
        r = A @ ell
        assert np.abs(r[interior]).max() <= 1e-12


def test_load_sums_to_volume():
    m = W.kuhn_cube(7, 5)
    b = fem.load_const(m.xyz, m.tets, 1.0)
    assert abs(b.sum() - 1.0) <= 1e-13
    b3 = fem.load_const(m.xyz, m.tets, 3.0)
    np.testing.assert_allclose(b3, 3 * b, rtol=1e-15)


@pytest.mark.parametrize("s", [0, 1, 2])
def test_grundmann_moeller_degree(s):
    """Exact on every monomial of the barycentric coordinates up to degree
    2s+1 (Dirichlet integral: int_T prod lambda^a = 3! prod a! / (3+|a|)!
    |T|), inexact at degree 2s+2."""
    lam, w = fem.grundmann_moeller(s)
    assert abs(w.sum() - 1.0) <= 1e-13
    rng = np.random.default_rng(s)
    for deg in range(0, 2 * s + 3):
        errs = []
        for _ in range(6):
            a = rng.multinomial(deg, [0.25] * 4)
            exact = 6.0 * np.prod([factorial(k) for k in a]) / factorial(3 + deg)
            q = np.sum(w * np.prod(lam ** a[None, :], axis=1))
            errs.append(abs(q - exact) / exact)
        if deg <= 2 * s + 1:
            assert max(errs) <= 1e-12, (deg, errs)
        else:
            assert max(errs) > 1e-6, (deg, errs)


def test_kappa_special_values():
    c = np.array([[0.3, 0.4, 0.5]])
    kap = W.KappaField("loggauss", centres=c, mu=np.array([np.log(3.0)]), width=0.02)
    pts = np.array([[0.3, 0.4, 0.5], [5.0, 5.0, 5.0]])
    k = fem.kappa_eval(pts, kap)
    assert abs(k[0] - 3.0) <= 1e-14 and abs(k[1] - 1.0) <= 1e-15
    # one width away along an axis: exp(log3 * e^{-1/2}) with |x-c|^2 = width/2
    p = c + np.array([[np.sqrt(0.01), 0, 0]])
    assert abs(fem.kappa_eval(p, kap)[0] - 3.0 ** np.exp(-0.5)) <= 1e-14
    # amplitudes add in the exponent: two identical centres square kappa
    kap2 = W.KappaField("loggauss", centres=np.vstack([c, c]), mu=np.array([np.log(3.0)] * 2), width=0.02)
    assert abs(fem.kappa_eval(pts[:1], kap2)[0] - 9.0) <= 1e-13


def test_nested_galerkin_identity():
    """Un-jittered Kuhn n inside 2n is nested (Freudenthal refinement), so
    P^T A_2n P == A_n for the unconstrained matrices, kappa = 1."""
    from oracle import transfer

    for n in (2, 3):
        c = W.kuhn_cube(n)
        f = W.kuhn_cube(2 * n)
        P = transfer.interpolation(f, c, mask_dirichlet=False, locate=transfer.locate_bruteforce)
        Af = fem.stiffness_neumann(f.xyz, f.tets, W.KappaField())
        Ac = fem.stiffness_neumann(c.xyz, c.tets, W.KappaField())
        G = (P.T @ Af @ P).toarray()
        assert np.abs(G - Ac.toarray()).max() <= 1e-13


@pytest.mark.slow
def test_l2_error_second_order():
    """u = sin(pi x) sin(pi y) sin(pi z), kappa = 1, f = 3 pi^2 u: the FE L2
    error shrinks as O(h^2) on jittered meshes."""
    u = lambda p: np.sin(np.pi * p[:, 0]) * np.sin(np.pi * p[:, 1]) * np.sin(np.pi * p[:, 2])
    f = lambda p: 3 * np.pi ** 2 * u(p)
    errs = []
    ns = [8, 16, 32]
    for n in ns:
        m = W.kuhn_cube(n, 1000 + n)
        A_N = fem.stiffness_neumann(m.xyz, m.tets, W.KappaField())
        b = fem.load_quadrature(m.xyz, m.tets, f, s=2)
        A, b = fem.dirichlet_eliminate(A_N, b, m.dirichlet)
        x = spla.spsolve(A.tocsc(), b)
        errs.append(fem.l2_error(m.xyz, m.tets, x, u, s=2))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates >= 1.8), (errs, rates)


def test_per_tet_load_is_the_exact_integral():
    """f constant per element: b_a = sum f_T |T| / 4 equals a constant f's load
    when all values agree, and the quadrature of the element-wise constant
    function (the rule, pinned by its exactness above, integrates lambda_a
    exactly)."""
    m = W.kuhn_cube(5, 21)
    assert np.abs(fem.load_per_tet(m.xyz, m.tets, np.full(m.nt, 2.5)) - fem.load_const(m.xyz, m.tets, 2.5)).max() \
        <= 1e-16
    fT = np.random.default_rng(4).uniform(-3, 3, m.nt)
    bq = fem.load_quadrature(m.xyz, m.tets, lambda p: fT, s=1)
    b = fem.load_per_tet(m.xyz, m.tets, fT)
    assert np.abs(b - bq).max() <= 1e-15 * np.abs(bq).max() * 10


def test_nodal_load_is_the_exact_integral_of_the_interpolant():
    """b = M f for P1 nodal values: constant values give the constant load,
    and for a linear f (which its P1 interpolant reproduces) the load equals
    the degree-3 quadrature of f lambda_a entry by entry -- this fixes the
    element mass matrix |T| (1 + delta_ab) / 20."""
    m = W.kuhn_cube(5, 22)
    assert np.abs(fem.load_nodal(m.xyz, m.tets, np.full(m.nv, -1.5)) - fem.load_const(m.xyz, m.tets, -1.5)).max() \
        <= 1e-16
    lin = lambda p: 0.7 - 2.0 * p[:, 0] + 3.5 * p[:, 1] + 1.25 * p[:, 2]
    b = fem.load_nodal(m.xyz, m.tets, lin(m.xyz))
    bq = fem.load_quadrature(m.xyz, m.tets, lin, s=1)
    assert np.abs(b - bq).max() <= 1e-14 * np.abs(bq).max()
    # a quadratic is not reproduced: the nodal load then differs
    quad = lambda p: p[:, 0] ** 2
    assert np.abs(fem.load_nodal(m.xyz, m.tets, quad(m.xyz)) - fem.load_quadrature(m.xyz, m.tets, quad, s=1)).max() \
        > 1e-6


@pytest.mark.slow
def test_l2_error_second_order_nodal_load():
    """The same O(h^2) rate with the load of the P1 interpolant of f
    (nodal values), the form the library takes for a general f."""
    u = lambda p: np.sin(np.pi * p[:, 0]) * np.sin(np.pi * p[:, 1]) * np.sin(np.pi * p[:, 2])
    errs = []
    for n in [8, 16, 32]:
        m = W.kuhn_cube(n, 1000 + n)
        A, b = fem.assemble(m, W.KappaField(), W.LoadField("nodal", 3 * np.pi ** 2 * u(m.xyz)))
        x = spla.spsolve(A.tocsc(), b)
        errs.append(fem.l2_error(m.xyz, m.tets, x, u, s=2))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates >= 1.8), (errs, rates)


def test_per_level_kappa_arrays_in_the_hierarchy():
    """Per-tetrahedron kappa given per level equals the field evaluated at
    each level's own centroids (the oracle's hierarchy takes either)."""
    from oracle import problem

    pb = W.Problem("t", [W.kuhn_cube(6, 1), W.kuhn_cube(3, 2)], [2], W.kappa_draw(204, 205))
    arrs = [fem.kappa_eval(fem.tet_geometry(m.xyz, m.tets)[2], pb.kappa) for m in pb.meshes]
    pb2 = W.Problem("t", pb.meshes, [2], W.KappaField("per_tet", value=arrs))
    h1, h2 = problem.build(pb), problem.build(pb2)
    for A1, A2 in zip(h1.A, h2.A):
        assert (A1 != A2).nnz == 0

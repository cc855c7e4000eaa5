"""Pins of the oracle's P1 linear elasticity and field-split interpolation
(Section 4.2's equations, Section 3.2's equation interpolation split), no
GPU: the six rigid motions span the null space of the Neumann matrix for any
E field, linear displacements pass the patch test, a manufactured solution
converges at second order (this fixes the roles of lambda and mu), the
split interpolation reproduces linear vector fields and satisfies the nested
Galerkin identity per field, and the multilevel solve reaches x*."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import elasticity as el, fem, problem, transfer


def test_lame_coefficients():
    mu, lam = el.lame(2.1e3, 0.25)
    assert abs(mu - 840.0) <= 1e-12 and abs(lam - 840.0) <= 1e-12  # nu = 1/4: lambda = mu = E / 2.5
    D = el.voigt_stiffness(1.0, 0.0)
    assert np.allclose(D, np.diag([1, 1, 1, 0.5, 0.5, 0.5]))


@pytest.mark.parametrize("seed", [3, 4])
def test_rigid_motions_are_the_null_space(seed):
    m = W.kuhn_cube(4, seed)
    E = fem.kappa_eval(fem.tet_geometry(m.xyz, m.tets)[2], W.kappa_draw(204, 205))
    A = el.stiffness_neumann(m.xyz, m.tets, E, 0.3)
    assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
    R = el.rigid_modes(m.xyz)
    for r in R:
        assert np.abs(A @ r).max() <= 1e-12 * abs(A).max()
    # exactly six: the seventh smallest eigenvalue is well away from zero
    w = np.linalg.eigvalsh(A.toarray())
    assert np.all(np.abs(w[:6]) <= 1e-10 * w[-1]) and w[6] > 1e-4 * w[-1]


def test_patch_test_linear_displacement():
    m = W.kuhn_cube(5, 8)
    A = el.stiffness_neumann(m.xyz, m.tets, 3.0, 0.35)
    G = np.array([[0.3, -1.2, 0.5], [0.7, 0.1, -0.4], [-0.9, 0.6, 1.1]])
    u = (m.xyz @ G.T + np.array([0.2, -0.1, 0.4])).ravel()
    r = A @ u
    inner = el.dof_mask(m.dirichlet) == 0
    assert np.abs(r[inner]).max() <= 1e-12 * abs(A).max()


def _manufactured(mu, lam):
    a = np.array([1.0, 0.5, -0.75])
    pi = np.pi

    def s_hess(p):
        x, y, z = p[:, 0], p[:, 1], p[:, 2]
        sx, sy, sz = np.sin(pi * x), np.sin(pi * y), np.sin(pi * z)
        cx, cy, cz = np.cos(pi * x), np.cos(pi * y), np.cos(pi * z)
        s = sx * sy * sz
        H = np.empty((p.shape[0], 3, 3))
        H[:, 0, 0] = H[:, 1, 1] = H[:, 2, 2] = -pi * pi * s
        H[:, 0, 1] = H[:, 1, 0] = pi * pi * cx * cy * sz
        H[:, 0, 2] = H[:, 2, 0] = pi * pi * cx * sy * cz
        H[:, 1, 2] = H[:, 2, 1] = pi * pi * sx * cy * cz
        return s, H

    def u(p, c):
        return a[c] * s_hess(p)[0]

    def f(p, c):
        # -div sigma = -mu lap u - (lambda + mu) grad div u, u = a s
        s, H = s_hess(p)
        return 3 * pi * pi * mu * a[c] * s - (lam + mu) * (H[:, c, :] @ a)

    return u, f


@pytest.mark.slow
def test_manufactured_solution_second_order():
    E, nu = 2.0, 0.3
    mu, lam = el.lame(E, nu)
    u, f = _manufactured(mu, lam)
    errs = []
    ns = (8, 16, 24)
    for n in ns:
        m = W.kuhn_cube(n, 2000 + n)
        A_N = el.stiffness_neumann(m.xyz, m.tets, E, nu)
        b = np.zeros(3 * m.nv)
        for c in range(3):
            b[c::3] = fem.load_quadrature(m.xyz, m.tets, lambda p: f(p, c), s=2)
        A, b = fem.dirichlet_eliminate(A_N, b, el.dof_mask(m.dirichlet))
        x = spla.splu(A.tocsc()).solve(b)
        e2 = sum(fem.l2_error(m.xyz, m.tets, x[c::3], lambda p: u(p, c), s=2) ** 2 for c in range(3))
        errs.append(np.sqrt(e2))
    rates = np.log(np.array(errs[:-1]) / np.array(errs[1:])) / np.log(np.array(ns[1:]) / np.array(ns[:-1]))
    assert np.all(rates >= 1.8), (errs, rates)


def test_split_interpolation_reproduces_linear_vector_fields():
    fine, coarse = W.kuhn_cube(7, 31), W.kuhn_cube(4, 32)
    P = transfer.interpolation(fine, coarse, mask_dirichlet=False, locate=transfer.locate_bruteforce)
    I = el.split_interpolation(P)
    G = np.array([[1.0, 2.0, -1.0], [0.5, -0.3, 0.2], [0.0, 1.5, 0.7]])
    lin = lambda X: (X @ G.T + np.array([0.1, 0.2, 0.3])).ravel()
    assert np.abs(I @ lin(coarse.xyz) - lin(fine.xyz)).max() <= 1e-13
    # field by field it is the scalar operator, and fields do not mix
    for c in range(3):
        for d in range(3):
            blk = I[c::3, d::3]
            assert (abs(blk - P).max() if c == d else abs(blk).max()) <= 0.0


def test_split_nested_galerkin_identity():
    """Un-jittered Kuhn n inside 2n (nested), E constant: the split transfer
    gives P^T A_2n P = A_n for the elasticity matrices."""
    for n in (2, 3):
        c, f = W.kuhn_cube(n), W.kuhn_cube(2 * n)
        P = el.split_interpolation(transfer.interpolation(f, c, mask_dirichlet=False,
                                                          locate=transfer.locate_bruteforce))
        Af = el.stiffness_neumann(f.xyz, f.tets, 1.7, 0.3)
        Ac = el.stiffness_neumann(c.xyz, c.tets, 1.7, 0.3)
        assert abs(P.T @ Af @ P - Ac).max() <= 1e-13 * abs(Ac).max()


def test_multilevel_elasticity_converges():
    pb = W.Problem("el", [W.kuhn_cube(9, 41), W.kuhn_cube(5, 42), W.kuhn_cube(3, 43)], [4, 2],
                   W.kappa_draw(204, 205))
    h = el.build(pb, nu=0.3)
    res = problem.solve(h)
    xs = problem.exact(h)
    assert res.converged and np.linalg.norm(res.x - xs) <= 1e-7 * np.linalg.norm(xs)
    # each smoothed level is much better than one level alone: a few iterations
    assert res.iterations <= 15

"""Pins of the oracle's barycentric non-nested interpolation (no GPU)."""
import numpy as np
import pytest

import workloads as W
from oracle import transfer


@pytest.mark.parametrize("nf,nc,sf,sc", [(6, 3, 1, 2), (9, 4, 3, 4), (16, 6, 101, 102)])
def test_reproduces_linear_functions(nf, nc, sf, sc):
    f, c = W.kuhn_cube(nf, sf), W.kuhn_cube(nc, sc)
    P = transfer.interpolation(f, c, mask_dirichlet=False)
    for coef in ([0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0.7, -1.3, 2.1, 0.4]):
        gc = c.xyz @ np.array(coef[:3]) + coef[3]
        gf = f.xyz @ np.array(coef[:3]) + coef[3]
        assert np.abs(P @ gc - gf).max() <= 1e-13
    rs = np.asarray(P.sum(axis=1)).ravel()
    assert np.abs(rs - 1).max() <= 1e-13
    assert P.data.min() >= -1e-12 and P.data.max() <= 1 + 1e-12
    assert np.all(np.diff(P.indptr) <= 4)


def test_bucket_equals_bruteforce():
    f, c = W.kuhn_cube(5, 8), W.kuhn_cube(3, 9)
    t1, l1 = transfer.locate_bruteforce(c.xyz, c.tets, f.xyz)
    t2, l2 = transfer.locate_bucket(c.xyz, c.tets, f.xyz)
    assert np.array_equal(t1, t2)
    np.testing.assert_allclose(l1, l2, atol=1e-15)


def test_identical_meshes_give_identity():
    m = W.kuhn_cube(5, 21)
    P = transfer.interpolation(m, m).toarray()
    interior = m.dirichlet == 0
    D = np.diag(interior.astype(float))
    assert np.abs(P - D).max() <= 1e-12


def test_dirichlet_masking():
    f, c = W.kuhn_cube(7, 1), W.kuhn_cube(3, 2)
    P = transfer.interpolation(f, c)
    assert P[np.nonzero(f.dirichlet)[0]].nnz == 0
    Pd = P.toarray()
    assert np.all(Pd[:, c.dirichlet != 0] == 0)


def test_point_outside_is_an_error():
    c = W.kuhn_cube(2, 3)
    pts = np.array([[0.5, 0.5, 0.5], [1.5, 0.5, 0.5]])
    with pytest.raises(transfer.PointLocationError):
        transfer.locate_bruteforce(c.xyz, c.tets, pts)
    with pytest.raises(transfer.PointLocationError):
        transfer.locate_bucket(c.xyz, c.tets, pts)


def test_lowest_index_rule_on_shared_faces():
    """A point on a face shared by two tetrahedra is given to the lower id."""
    c = W.kuhn_cube(1)
    # centroid of the cell lies on the main diagonal, shared by all six
    t, lam = transfer.locate_bruteforce(c.xyz, c.tets, np.array([[0.5, 0.5, 0.5]]))
    assert t[0] == 0

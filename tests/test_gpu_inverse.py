"""Dense subdomain solves applied through inverse panels (NNMS_APPLY_INVERSE)
against the FP64 oracle, through the C ABI.

The panels X_p are pinned to their definition, the owned columns of the
inverse of the oracle's subdomain matrix A[S_p, S_p] in the documented local
order (overlap rows first, owned rows last on the smoothed levels; the whole
inverse on the coarsest level).  Computed from the LU factors by block
substitution, they carry the factor's rounding times the block condition
number (~1e3 on these blocks): 1e-11 of max |J_p^{-1}| in FP64, 1e-4 in FP32.
The smoother, V-cycle and solves then follow the bars of the sweep path:
1e-9 relative, within one FGMRES iteration of the oracle, x* to 1e-7.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import problem as oprob

pytestmark = pytest.mark.gpu


def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08981_amd import nnms

    return nnms


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


class Built:
    def __init__(self, pb, precision="fp64", dense_apply=None):
        nnms = _gpu()
        prec = nnms.MIXED if precision == "mixed" else nnms.FP64
        self.pb = pb
        self.meshes = [nnms.Mesh.from_workload(m) for m in pb.meshes]
        mode = nnms.INVERSE if dense_apply is None else dense_apply
        self.h = nnms.Hierarchy(self.meshes, pb.nparts, overlap=pb.overlap, its=pb.its, precision=prec,
                                dense_apply=mode)
        self.s = nnms.System(self.h, pb.kappa, 1.0)


def _tiny3():
    return W.Problem("tiny3", [W.kuhn_cube(13, 11), W.kuhn_cube(7, 12), W.kuhn_cube(4, 13)], [4, 2],
                     W.kappa_draw(204, 205))


@pytest.fixture(scope="module")
def cases():
    _say("[gpu] building 16^3 / 6^3 and 13^3 / 7^3 / 4^3 problems with inverse panels (fp64)")
    out = {}
    for name, pb in (("cube16", W.cube16_two_level()), ("tiny3", _tiny3())):
        out[name] = (Built(pb), oprob.build(pb))
    return out


def _local_order(S, owner, p, smoothed):
    if not smoothed:
        return np.asarray(S)
    S = np.asarray(S)
    mine = np.asarray(owner)[S] == p
    return np.concatenate([S[~mine], S[mine]])


@pytest.mark.parametrize("case,precision", [("cube16", "fp64"), ("tiny3", "fp64"), ("tiny3", "mixed")])
def test_panels_are_owned_columns_of_the_inverse(case, precision, cases):
    g, o = cases[case]
    if precision == "mixed":
        g = Built(g.pb, precision="mixed")
    nnms = _gpu()
    L = len(g.pb.meshes)
    for l in range(L):
        assert g.h.level_info(l).dense_apply == nnms.INVERSE
        owner, sets = g.h.partition(l)
        A = o.A[l].tocsr()
        tol = 1e-11 if (precision == "fp64" or l == L - 1) else 1e-4
        for p, S in enumerate(sets):
            order = _local_order(S, owner, p, l < L - 1)
            n = len(order)
            nv = n - int(np.count_nonzero(np.asarray(owner)[order] == p)) if l < L - 1 else 0
            ref = np.linalg.inv(A[order][:, order].toarray())[:, nv:]
            X = g.s.inverse_panels(l, p)
            assert X.shape[0] % 64 == 0 and X.shape[0] >= n and X.shape[1] >= n - nv
            err = np.abs(X[:n, :n - nv] - ref).max() / np.abs(ref).max()
            assert err <= tol, (case, precision, l, p, err)
            assert not X[n:].any() and not X[:, n - nv:].any(), (l, p)
    if precision == "mixed":
        g.s.destroy()
        g.h.destroy()


@pytest.mark.parametrize("case", ["cube16", "tiny3"])
def test_smoother_vcycle_and_solve(case, cases):
    g, o = cases[case]
    rng = np.random.default_rng(2)
    L = len(g.pb.meshes)
    for l in range(L):
        r = rng.standard_normal(g.s.n[l])
        r[g.pb.meshes[l].dirichlet != 0] = 0
        z = g.s.apply_smoother(l, r)
        ref = o.vcycle.levels[l].ras.apply(r) if l < L - 1 else np.linalg.solve(o.A[l].toarray(), r)
        assert _rel(z, ref) <= 1e-9, (l, _rel(z, ref))
    r = rng.standard_normal(g.s.n[0])
    r[g.pb.meshes[0].dirichlet != 0] = 0
    assert _rel(g.s.apply_vcycle(r), o.vcycle(r)) <= 1e-9
    ref = oprob.solve(o)
    xs = oprob.exact(o)
    for graph in (True, False):
        x, info = g.s.solve(o.b, graph=graph)
        assert info.status == 0 and info.relres <= 1e-8
        assert abs(info.iterations - ref.iterations) <= 1, (info.iterations, ref.iterations)
        assert _rel(x, xs) <= 1e-7


def test_mixed_precision_solve():
    pb = _tiny3()
    g = Built(pb, precision="mixed")
    o = oprob.build(pb)
    x, info = g.s.solve(o.b)
    assert info.status == 0 and info.relres <= 1e-8
    ref = oprob.solve(o)
    assert info.iterations <= ref.iterations + max(1, int(0.1 * ref.iterations) + 1)
    assert _rel(x, oprob.exact(o)) <= 1e-7


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_of_both_modes_equals_alone(precision):
    """Systems applying their dense solves by sweeps and by inverse panels,
    on different meshes and subdomain counts, in one batch: every slot gets
    the bits of its solve alone, and the oracle's solution."""
    nnms = _gpu()
    prec = nnms.MIXED if precision == "mixed" else nnms.FP64
    keep, systems, bs, xstar = [], [], [], []
    for i, (n, nps, mode) in enumerate([(9, [2, 2], nnms.INVERSE), (12, [4, 2], nnms.SWEEPS),
                                         (14, [8, 2], nnms.INVERSE), (10, [2, 2], nnms.SWEEPS)]):
        ns = W.coarse_sizes(n)
        pb = W.Problem(f"m{i}", W.make_hierarchy(ns, [900 + 10 * i + l for l in range(3)]), nps,
                       W.kappa_draw(204, 909 + 10 * i), precision=precision)
        ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
        h = nnms.Hierarchy(ms, pb.nparts, precision=prec, dense_apply=mode)
        s = nnms.System(h, pb.kappa)
        o = oprob.build(pb)
        keep.append((ms, h))
        systems.append(s)
        bs.append(o.b)
        xstar.append(oprob.exact(o))
    alone = [s.solve(b) for s, b in zip(systems, bs)]
    xs, infos = nnms.solve_batch(systems, bs, graph=True)
    for k in range(len(systems)):
        assert np.array_equal(xs[k], alone[k][0]), k
        assert infos[k].iterations == alone[k][1].iterations
        assert infos[k].status == 0 and infos[k].relres <= 1e-8
        assert _rel(xs[k], xstar[k]) <= 1e-7


def test_refactoring_in_place_gives_the_same_panels(cases):
    """A new assembly of the same parameter (the numeric setup again, in
    place) reproduces the panels bit for bit."""
    g, _ = cases["tiny3"]
    before = [g.s.inverse_panels(0, p) for p in range(g.h.level_info(0).nparts)]
    g.s.time_kernel(6, 0, reps=1)
    for p, X in enumerate(before):
        assert np.array_equal(g.s.inverse_panels(0, p), X), p


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_direct_level(precision):
    """One level only: the whole system is the coarsest level, solved through
    its whole inverse.  9,261 unknowns (145 tiles per side) are more rows
    than the smoother stages in LDS, so its work items read the gathered
    rows from global memory instead: the direct solve against a sparse
    direct solve, entry by entry (1e-10 relative in FP64; 2e-5 in mixed
    precision, whose level vectors are FP32: their rounding times the
    condition number), and one FGMRES iteration (two in mixed precision)."""
    import scipy.sparse.linalg as spla

    nnms = _gpu()
    from oracle import fem

    mesh = W.kuhn_cube(22, 77)
    pb = W.Problem("direct22", [mesh], [], W.kappa_draw(204, 205), precision=precision)
    g = Built(pb, precision=precision)
    li = g.h.level_info(0)
    assert li.dense_apply == nnms.INVERSE and (li.ninterior + 63) // 64 > 128
    A, b = fem.assemble(mesh, pb.kappa)
    r = np.random.default_rng(21).standard_normal(mesh.nv)
    r[mesh.dirichlet != 0] = 0
    z = g.s.apply_smoother(0, r)
    ref = spla.spsolve(A.tocsc(), r)
    tol = 1e-10 if precision == "fp64" else 2e-5
    assert np.abs(z - ref).max() <= tol * np.abs(ref).max()
    x, info = g.s.solve(b)
    assert info.status == 0 and info.relres <= 1e-8 and info.iterations <= (1 if precision == "fp64" else 2)


@pytest.mark.parametrize("overlap", [0, 1, 2])
def test_tiny_and_ragged_subdomains(overlap):
    """Subdomains smaller than one tile (9^3 fine mesh in 16 parts: 32 owned
    rows), no overlap (every subdomain its own whole inverse, lower triangle
    only, no overlap part) and two layers (more overlap rows than owned
    ones): panels, smoother and V-cycle against the oracle, and a solve."""
    pb = W.Problem("tiny", [W.kuhn_cube(9, 31), W.kuhn_cube(5, 32), W.kuhn_cube(3, 33)], [16, 4],
                   W.kappa_draw(204, 205), overlap=overlap)
    g = Built(pb)
    o = oprob.build(pb)
    L = len(pb.meshes)
    for l in range(L):
        owner, sets = g.h.partition(l)
        A = o.A[l].tocsr()
        for p, S in enumerate(sets):
            order = _local_order(S, owner, p, l < L - 1)
            n = len(order)
            nv = n - int(np.count_nonzero(np.asarray(owner)[order] == p)) if l < L - 1 else 0
            ref = np.linalg.inv(A[order][:, order].toarray())[:, nv:]
            X = g.s.inverse_panels(l, p)
            assert np.abs(X[:n, :n - nv] - ref).max() <= 1e-11 * np.abs(ref).max(), (l, p)
        rng = np.random.default_rng(40 + l)
        r = rng.standard_normal(g.s.n[l])
        r[pb.meshes[l].dirichlet != 0] = 0
        z = g.s.apply_smoother(l, r)
        ref = o.vcycle.levels[l].ras.apply(r) if l < L - 1 else np.linalg.solve(o.A[l].toarray(), r)
        assert _rel(z, ref) <= 1e-9, (l, _rel(z, ref))
    r = np.random.default_rng(3).standard_normal(g.s.n[0])
    r[pb.meshes[0].dirichlet != 0] = 0
    assert _rel(g.s.apply_vcycle(r), o.vcycle(r)) <= 1e-9
    x, info = g.s.solve(o.b)
    assert info.status == 0 and info.relres <= 1e-8
    assert abs(info.iterations - oprob.solve(o).iterations) <= 1

"""Parity of the ILU(k) subdomain solver of the smoother (Section 4 runs RAS
with ILU(p) subdomain solves) on the HIP path with the FP64 oracle, through
the C ABI.

Tolerances: the factorisation performs the same operations in the same
order as the oracle's (row by row, eliminations in ascending column order),
so the factors agree to a few ulps of the matrix scale (1e-12 of max |A|);
the triangular solves sum in another order than SciPy's, and smoother,
V-cycle and solve outputs are compared to 1e-10 relative; solves reach
relres <= 1e-8 within one step of the oracle's iteration count.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import fem, ilu, problem as oprob

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
    def __init__(self, pb, fill, precision=None, subsolver=None, transfer=None):
        nnms = _gpu()
        prec = nnms.MIXED if (precision or pb.precision) == "mixed" else nnms.FP64
        self.pb = pb
        self.fill = fill
        self.meshes = [nnms.Mesh.from_workload(m) for m in pb.meshes]
        self.h = nnms.Hierarchy(self.meshes, pb.nparts, overlap=pb.overlap, its=pb.its, precision=prec,
                                subsolver=nnms.ILU if subsolver is None else subsolver, ilu_fill=fill,
                                transfer=nnms.BARYCENTRIC if transfer is None else transfer)
        self.s = nnms.System(self.h, pb.kappa, 1.0)


def _tiny3(precision="fp64"):
    return W.Problem("tiny3", [W.kuhn_cube(13, 11), W.kuhn_cube(7, 12), W.kuhn_cube(4, 13)], [4, 2],
                     W.kappa_draw(204, 205), precision=precision)


@pytest.fixture(scope="module")
def tiny3i():
    _say("[gpu] ILU(2)/ILU(0) smoother: ragged 3-level case 13^3 / 7^3 / 4^3 (fp64)")
    pb = _tiny3()
    return Built(pb, [2, 0]), oprob.build(pb, ilu_fill=[2, 0])


@pytest.fixture(scope="module")
def cube16i():
    _say("[gpu] ILU(0) smoother: two-level 16^3 / 6^3 problem (fp64)")
    pb = W.cube16_two_level()
    return Built(pb, [0]), oprob.build(pb, ilu_fill=[0])


def _check_factors(g, o, level, parts=None):
    rp, col = g.h.ilu_pattern(level)
    val = g.s.ilu_values(level)
    owner, sets = g.h.partition(level)
    A = o.A[level]
    scale = abs(A).max()
    row = 0
    for p, S in enumerate(sets):
        n = len(S)
        if parts is None or p in parts:
            ras = o.vcycle.levels[level].ras
            f = ras.lu[p]
            L, U = f.L.tocsr(), f.U.tocsr()
            for i in range(n):
                a, b = rp[row + i], rp[row + i + 1]
                cols = col[a:b]
                ref = np.array([L[i, j] if j < i else U[i, j] for j in cols])
                assert np.abs(val[a:b] - ref).max() <= 1e-12 * scale, (level, p, i)
        row += n


@pytest.mark.parametrize("case", ["tiny3i", "cube16i"])
def test_factors_match_oracle(case, request):
    g, o = request.getfixturevalue(case)
    for l in range(len(g.pb.meshes) - 1):
        _check_factors(g, o, l)


@pytest.mark.parametrize("case", ["tiny3i", "cube16i"])
def test_smoother_and_vcycle_match_oracle(case, request):
    g, o = request.getfixturevalue(case)
    rng = np.random.default_rng(21)
    for l in range(len(g.pb.meshes) - 1):
        r = rng.standard_normal(g.s.n[l])
        r[g.pb.meshes[l].dirichlet != 0] = 0
        assert _rel(g.s.apply_smoother(l, r), o.vcycle.levels[l].ras.apply(r)) <= 1e-10, l
    r = rng.standard_normal(g.s.n[0])
    r[g.pb.meshes[0].dirichlet != 0] = 0
    assert _rel(g.s.apply_vcycle(r), o.vcycle(r)) <= 1e-10


@pytest.mark.parametrize("case", ["tiny3i", "cube16i"])
@pytest.mark.parametrize("graph", [True, False])
def test_solve_matches_oracle(case, graph, request):
    g, o = request.getfixturevalue(case)
    ref = oprob.solve(o)
    x, info = g.s.solve(o.b, graph=graph)
    assert info.status == 0 and info.relres <= 1e-8
    assert abs(info.iterations - ref.iterations) <= 1
    assert np.linalg.norm(o.b - o.A[0] @ x) <= 1e-8 * np.linalg.norm(o.b)
    assert _rel(x, oprob.exact(o)) <= 1e-7
    x2, info2 = g.s.solve(o.b, graph=graph)
    assert np.array_equal(x, x2) and info2.iterations == info.iterations


def test_mixed_precision_ilu():
    pb = _tiny3("mixed")
    g = Built(pb, [2, 0])
    o = oprob.build(pb, ilu_fill=[2, 0])
    x, info = g.s.solve(o.b)
    ref = oprob.solve(o)
    assert info.status == 0 and info.relres <= 1e-8
    assert info.iterations <= int(np.ceil(1.1 * ref.iterations)) + 1
    assert _rel(x, oprob.exact(o)) <= 1e-7
    # FP32 factors: the same elimination, rounded to FP32
    rp, col = g.h.ilu_pattern(0)
    val = g.s.ilu_values(0)
    owner, sets = g.h.partition(0)
    f = o.vcycle.levels[0].ras.lu[0]
    L, U = f.L.tocsr(), f.U.tocsr()
    scale = abs(o.A[0]).max()
    for i in range(len(sets[0])):
        a, b = rp[i], rp[i + 1]
        ref = np.array([L[i, j] if j < i else U[i, j] for j in col[a:b]])
        assert np.abs(val[a:b] - ref).max() <= 1e-4 * scale


def test_batch_of_ilu_and_dense_systems_equals_alone(tiny3i):
    nnms = _gpu()
    g1, o1 = tiny3i
    g2 = Built(_tiny3(), [0, 0])
    g3 = Built(_tiny3(), [2, 0], subsolver=nnms.LU)
    g4 = Built(_tiny3(), [1, 1], transfer=nnms.MLS)
    alone = [g.s.solve(o1.b) for g in (g1, g2, g3, g4)]
    xs, infos = nnms.solve_batch([g1.s, g2.s, g3.s, g4.s], [o1.b] * 4)
    for (x, i), xb, ib in zip(alone, xs, infos):
        assert np.array_equal(xb, x) and ib.iterations == i.iterations


def test_autotune_on_ilu_levels_keeps_results(tiny3i):
    """The autotuner times only the launches a level has: on ILU levels it
    leaves the dense smoother's shape alone (regression: it once launched
    the dense smoother over an ILU level's absent dense factors)."""
    nnms = _gpu()
    from paper_2412_08981_amd import autotune

    pb = _tiny3()
    g = Built(pb, [2, 0])
    o = tiny3i[1]
    x0, i0 = g.s.solve(o.b)
    before = g.h.get_tuning()
    t = autotune.tune(g.s, cache=None, reps=2)
    assert t["ras_blocks"][0] == before["ras_blocks"][0] and t["ras_blocks"][1] == before["ras_blocks"][1]
    x1, i1 = g.s.solve(o.b)
    assert i1.iterations == i0.iterations and _rel(x1, x0) <= 1e-10


def test_one_subdomain_full_fill_is_exact():
    """One subdomain, no overlap, fill level above the matrix size: nothing
    is dropped, so the smoother is the exact inverse."""
    nnms = _gpu()
    pb = W.Problem("exact", [W.kuhn_cube(4, 41), W.kuhn_cube(2, 42)], [1], W.kappa_draw(1, 2), overlap=0)
    g = Built(pb, [64])
    o = oprob.build(pb)
    r = np.random.default_rng(5).standard_normal(g.s.n[0])
    r[pb.meshes[0].dirichlet != 0] = 0
    z = g.s.apply_smoother(0, r)
    assert _rel(o.A[0] @ z, r) <= 1e-12


def test_dense_readback_is_refused_on_ilu_levels(cube16i):
    nnms = _gpu()
    g, o = cube16i
    with pytest.raises(nnms.NNMSError):
        g.s.factor(0, 0)


def test_full_size_ilu2_ilu0():
    """48^3 / 24^3 / 10^3 with ILU(2) on the fine level and ILU(0) on the
    second (the paper's setting): one subdomain per level against the
    oracle's factorisation, and a solve to the true relative residual 1e-8."""
    nnms = _gpu()
    _say("[gpu] ILU(2)/ILU(0) smoother: 48^3 / 24^3 / 10^3 three-level problem (fp64)")
    pb = W.cube48_three_level()
    g = Built(pb, [2, 0])
    rng = np.random.default_rng(23)
    for l, fill in ((0, 2), (1, 0)):
        A, _ = fem.assemble(pb.meshes[l], pb.kappa)
        owner, sets = g.h.partition(l)
        p = int(rng.integers(len(sets)))
        S = sets[p]
        f = ilu.ILU(A[S][:, S].tocsr(), fill)
        L, U = f.L.tocsr(), f.U.tocsr()
        rp, col = g.h.ilu_pattern(l)
        val = g.s.ilu_values(l)
        base = sum(len(sets[q]) for q in range(p))
        scale = abs(A).max()
        for i in range(0, len(S), 7):
            a, b = rp[base + i], rp[base + i + 1]
            assert np.array_equal(col[a:b], f.cols[i]), (l, i)
            ref = np.array([L[i, j] if j < i else U[i, j] for j in col[a:b]])
            assert np.abs(val[a:b] - ref).max() <= 1e-12 * scale, (l, i)
    # the true residual from the oracle's assembly
    A0, b = fem.assemble(pb.meshes[0], pb.kappa)
    x, info = g.s.solve(b)
    assert info.status == 0 and info.relres <= 1e-8
    assert np.linalg.norm(b - A0 @ x) <= 1e-8 * np.linalg.norm(b)
    _say(f"[gpu] ILU(2)/ILU(0) at 48^3: {info.iterations} iterations")

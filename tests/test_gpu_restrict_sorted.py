"""The restriction P_l^T in column-sorted slices (tuning value pt_lanes = 2:
64 coarse rows per slice, the slice's entries stored in fine-column order,
the products regrouped by row in LDS).  It is the same product as the CSR
kernels with the row sums in another order, so:

* every entry of the device product against the oracle's P_l^T x on a
  ragged three-level case (coarse levels of 1,000 and 125 vertices: 16 and
  2 slices, the last ones partial), FP64 to 1e-13 of max |ref|, FP32 to
  2e-6 (the inputs and products rounded to FP32, ~30 terms per row), and
  against the CSR kernel's product on the same data (FP64, 1e-14);
* a solve through it equal to the default shapes' to rounding, with the
  same iteration count;
* at the benchmark's 48^3 size, every entry against the oracle (1e-13);
* on the largest served hierarchy (96^3 fine level, 117,649 coarse rows),
  every entry against the product of the stored P_l^T (the stored matrix
  equals the oracle's entry by entry at 48^3, where the oracle's point
  location is cheap enough to run in a test);
* in a batch beside systems with other shapes every slot keeps its bits
  alone.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import problem as oprob

pytestmark = pytest.mark.gpu
CSORT = 2


def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08981_amd import nnms

    return nnms


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _close(v, ref, tol):
    """Entry-wise agreement: max |v - ref| <= tol max |ref|."""
    return float(np.abs(v - ref).max()) <= tol * max(float(np.abs(ref).max()), 1e-300)


def _err(v, ref):
    return float(np.abs(v - ref).max()) / max(float(np.abs(ref).max()), 1e-300)


def _interior_random(rng, mesh):
    r = rng.standard_normal(mesh.nv)
    r[mesh.dirichlet != 0] = 0
    return r


def _with_pt(nnms, h, pb, g):
    d = h.get_tuning()
    d["pt_lanes"] = [g] * len(d["pt_lanes"])
    h.set_tuning(d)
    return nnms.System(h, pb.kappa, 1.0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sorted_restriction_matches_oracle(precision):
    nnms = _gpu()
    _say(f"[gpu] column-sorted P^T on 17^3 / 9^3 / 4^3 ({precision})")
    pb = W.Problem("csort", W.make_hierarchy([17, 9, 4], [61, 62, 63]), [4, 2], W.kappa_draw(204, 207),
                   precision=precision)
    prec = nnms.MIXED if precision == "mixed" else nnms.FP64
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, precision=prec)
    o = oprob.build(pb)
    s0 = nnms.System(h, pb.kappa, 1.0)
    x0, i0 = s0.solve(o.b)
    s16 = _with_pt(nnms, h, pb, 16)
    s = _with_pt(nnms, h, pb, CSORT)
    assert h.get_tuning()["pt_lanes"][0] == CSORT
    rng = np.random.default_rng(8)
    tol = 1e-13 if precision == "fp64" else 2e-6
    for l in range(2):
        x = _interior_random(rng, pb.meshes[l])
        y = s.apply_restrict(l, x)
        ref = o.P[l].T @ x
        assert _close(y, ref, tol), (l, _err(y, ref))
        if precision == "fp64":
            y16 = s16.apply_restrict(l, x)
            assert _close(y, y16, 1e-14), (l, _err(y, y16))
        assert np.array_equal(y, s.apply_restrict(l, x))  # deterministic
    x1, i1 = s.solve(o.b)
    assert i1.status == 0 and i1.relres <= 1e-8 and i1.iterations == i0.iterations
    assert np.linalg.norm(x1 - x0) <= (1e-10 if precision == "fp64" else 1e-6) * np.linalg.norm(x0)
    for sy in (s, s16, s0):
        sy.destroy()


def test_sorted_restriction_full_size_48():
    nnms = _gpu()
    _say("[gpu] column-sorted P^T at 48^3 / 24^3 / 10^3 (fp64)")
    pb = W.cube48_three_level("fp64")
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, overlap=pb.overlap, its=pb.its)
    o = oprob.build(pb)
    s = _with_pt(nnms, h, pb, CSORT)
    rng = np.random.default_rng(9)
    for l in range(2):
        x = _interior_random(rng, pb.meshes[l])
        y = s.apply_restrict(l, x)
        ref = o.P[l].T @ x
        assert _close(y, ref, 1e-13), (l, _err(y, ref))
    s.destroy()


def test_sorted_restriction_served_96():
    nnms = _gpu()
    _say("[gpu] column-sorted P^T on the served 96^3 / 48^3 / 20^3 hierarchy (fp64)")
    meshes = W.served_hierarchy(96)
    nps = [W.nparts_rule(m.nv) for m in meshes[:-1]]
    pb = W.Problem("served96", meshes, nps, W.kappa_draw(5003, 5004))
    ms = [nnms.Mesh.from_workload(m) for m in meshes]
    h = nnms.Hierarchy(ms, nps)
    s = _with_pt(nnms, h, pb, CSORT)
    rng = np.random.default_rng(10)
    for l in range(2):
        rp, col, w = h.restriction_csr(l)
        R = sp.csr_matrix((w, col, rp), shape=(s.n[l + 1], s.n[l]))
        x = _interior_random(rng, meshes[l])
        y = s.apply_restrict(l, x)
        ref = R @ x
        assert _close(y, ref, 1e-13), (l, _err(y, ref))
    s.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sorted_restriction_batch_same_bits(precision):
    nnms = _gpu()
    prec = nnms.MIXED if precision == "mixed" else nnms.FP64
    keep, systems, bs, alone = [], [], [], []
    for n, gp, seed in ((15, CSORT, 71), (13, 16, 81), (14, CSORT, 91), (12, 0, 101)):
        pb = W.Problem("b", W.make_hierarchy([n, n // 2, 3], [seed, seed + 1, seed + 2]), [4, 2],
                       W.kappa_draw(204, seed))
        ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
        h = nnms.Hierarchy(ms, pb.nparts, precision=prec)
        s = _with_pt(nnms, h, pb, gp)
        b = s.rhs()
        keep.append((ms, h))
        systems.append(s)
        bs.append(b)
        alone.append(s.solve(b))
    xs, infos = nnms.solve_batch(systems, bs)
    for k, (x, info) in enumerate(alone):
        assert infos[k].iterations == info.iterations
        assert np.array_equal(xs[k], x), k

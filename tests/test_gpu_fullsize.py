"""The default path (dense subdomain LU, barycentric transfer) at the
benchmark's full size and launch configuration (the tuned shapes of the
committed cache), against the FP64 oracle, entry by entry.

A vector v is compared with the oracle's r entry-wise: max_i |v_i - r_i| <=
tol * max_i |r_i|.  48^3 / 24^3 / 10^3, 64 + 32 subdomains: the assembled
operators, the load vector, every entry of P_l and P_l^T as stored, and the
device products with them (the same sums in another order, 1e-13); the
smoother on every level, all subdomains at once, against the oracle's
restricted additive Schwarz with LAPACK (1e-9: rounding times the blocks'
condition numbers), the coarsest direct solve, one V-cycle against the
oracle's V-cycle (1e-9), and a full FP64 solve against the oracle's own FGMRES
solution (same iteration count within one, 1e-7).  Mixed precision: the FP32
smoother on both levels against the oracle's (1e-2: FP32 rounding times block
condition numbers up to ~1e5) and a solve against x* (1e-7).  The same
smoother, V-cycle and solve checks with the dense solves applied through
inverse panels (the benchmark's default), in both precisions.  96^3 / 48^3 /
20^3 (the largest served hierarchy, 512 fine subdomains, mixed): the true
residual of a solve from the oracle's assembly, and eight subdomains of the
fine smoother solved one by one by LAPACK.  The 32 batched instances: true
residuals and bitwise equality with solves alone.
"""
import os
import sys

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W
from oracle import fem, problem as oprob, schwarz

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.path.join(ROOT, "paper_2412_08981_amd", "tuning.json")


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


def _system(pb, precision, dense_apply=None):
    nnms = _gpu()
    from paper_2412_08981_amd import autotune

    prec = nnms.MIXED if precision == "mixed" else nnms.FP64
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, overlap=pb.overlap, its=pb.its, precision=prec,
                       dense_apply=nnms.SWEEPS if dense_apply is None else dense_apply)
    s = nnms.System(h, pb.kappa, 1.0)
    autotune.tune(s, cache=CACHE)  # the benchmark's launch shapes
    s.destroy()
    return nnms.System(h, pb.kappa, 1.0), h, ms


def _interior_random(rng, mesh):
    r = rng.standard_normal(mesh.nv)
    r[mesh.dirichlet != 0] = 0
    return r


def _check_smoother_samples(s, mesh, A, nparts, parts, tol):
    rng = np.random.default_rng(7)
    r = _interior_random(rng, mesh)
    z = s.apply_smoother(0, r)
    owned, sets = schwarz.partition(mesh, nparts, 1)
    for p in parts:
        S = sets[p]
        y = sla.lu_solve(sla.lu_factor(A[S][:, S].toarray()), r[S])
        own = np.sort(owned[p])
        ref = y[np.searchsorted(S, own)]
        assert _close(z[own], ref, tol), (p, _err(z[own], ref))


def _check_smoothers(s, pb, o, tol):
    """Every level's smoother, all subdomains, against the oracle's RAS (and
    the coarsest direct solve against numpy.linalg.solve)."""
    rng = np.random.default_rng(11)
    L = len(pb.meshes)
    for l in range(L):
        r = _interior_random(rng, pb.meshes[l])
        z = s.apply_smoother(l, r)
        ref = o.vcycle.levels[l].ras.apply(r) if l < L - 1 else np.linalg.solve(o.A[l].toarray(), r)
        assert _close(z, ref, tol), (l, _err(z, ref))


def test_cube48_fp64_full_size():
    _say("[gpu] 48^3 / 24^3 / 10^3 at the benchmark's launch shapes (fp64)")
    pb = W.cube48_three_level("fp64")
    s, h, keep = _system(pb, "fp64")
    o = oprob.build(pb)
    for l in range(3):
        rp, col = h.csr(l)
        A = sp.csr_matrix((s.matrix_values(l), col, rp), shape=(s.n[l], s.n[l]))
        assert abs(A - o.A[l]).max() <= 1e-13 * abs(o.A[l]).max(), l
    assert _close(s.rhs(), o.b, 1e-14)
    rng = np.random.default_rng(3)
    for l in range(2):
        # the stored operators, every entry
        rp, col, w = h.transfer_csr(l)
        P = sp.csr_matrix((w, col, rp), shape=o.P[l].shape)
        assert abs(P - o.P[l]).max() <= 1e-14, l
        rp, col, w = h.restriction_csr(l)
        R = sp.csr_matrix((w, col, rp), shape=o.P[l].T.shape)
        assert abs(R - o.P[l].T).max() <= 1e-14, l
        idx, wl = h.transfer(l)
        Pe = sp.csr_matrix((wl.ravel(), idx.ravel(), np.arange(0, 4 * s.n[l] + 1, 4)), shape=o.P[l].shape)
        assert abs(Pe - o.P[l]).max() <= 1e-14, l
        # the device products, every entry
        xc = rng.standard_normal(s.n[l + 1])
        assert _close(s.apply_prolong(l, xc), o.P[l] @ xc, 1e-13), l
        x = _interior_random(rng, pb.meshes[l])
        assert _close(s.apply_restrict(l, x), o.P[l].T @ x, 1e-13), l
        x = _interior_random(rng, pb.meshes[l])
        assert _close(s.apply_operator(l, x), o.A[l] @ x, 1e-13), l
    _check_smoothers(s, pb, o, 1e-9)
    r = _interior_random(rng, pb.meshes[0])
    zv = s.apply_vcycle(r)
    assert _close(zv, o.vcycle(r), 1e-9), _err(zv, o.vcycle(r))
    ref = oprob.solve(o)
    x, info = s.solve(o.b)
    _say(f"[gpu] 48^3 fp64: {info.iterations} iterations (oracle {ref.iterations})")
    assert info.status == 0 and info.relres <= 1e-8
    assert abs(info.iterations - ref.iterations) <= 1
    assert np.linalg.norm(o.b - o.A[0] @ x) <= 1e-8 * np.linalg.norm(o.b)
    assert _close(x, ref.x, 1e-7), _err(x, ref.x)


def test_cube48_mixed_full_size():
    _say("[gpu] 48^3 / 24^3 / 10^3 at the benchmark's launch shapes (mixed)")
    pb = W.cube48_three_level("mixed")
    s, h, keep = _system(pb, "mixed")
    o = oprob.build(pb)
    A, b = o.A[0], o.b
    x, info = s.solve(b)
    assert info.status == 0 and info.relres <= 1e-8
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    xs = oprob.exact(o)  # x* by a sparse direct solve
    assert _close(x, xs, 1e-7), _err(x, xs)
    # FP32 smoother, all subdomains of both levels: FP32 rounding (6e-8)
    # times the blocks' condition numbers (up to ~1e5 with this kappa)
    _check_smoothers(s, pb, o, 1e-2)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cube48_inverse_panels_full_size(precision):
    """The benchmark's default: dense subdomain solves through inverse
    panels, at the benchmark's size and launch configuration.  Every level's
    smoother (all subdomains) against the oracle's restricted additive
    Schwarz (FP64 1e-9; FP32 1e-2 as above), one V-cycle (FP64 1e-9), and a
    solve against the oracle's FGMRES solution (FP64: iterations within one,
    1e-7) or x* (mixed, 1e-7)."""
    nnms = _gpu()
    _say(f"[gpu] 48^3 / 24^3 / 10^3 with inverse panels ({precision})")
    pb = W.cube48_three_level(precision)
    s, h, keep = _system(pb, precision, nnms.INVERSE)
    assert all(h.level_info(l).dense_apply == nnms.INVERSE for l in range(3))
    o = oprob.build(pb)
    _check_smoothers(s, pb, o, 1e-9 if precision == "fp64" else 1e-2)
    rng = np.random.default_rng(5)
    x, info = s.solve(o.b)
    assert info.status == 0 and info.relres <= 1e-8
    assert np.linalg.norm(o.b - o.A[0] @ x) <= 1e-8 * np.linalg.norm(o.b)
    if precision == "fp64":
        r = _interior_random(rng, pb.meshes[0])
        zv = s.apply_vcycle(r)
        assert _close(zv, o.vcycle(r), 1e-9), _err(zv, o.vcycle(r))
        ref = oprob.solve(o)
        _say(f"[gpu] 48^3 inverse panels fp64: {info.iterations} iterations (oracle {ref.iterations})")
        assert abs(info.iterations - ref.iterations) <= 1
        assert _close(x, ref.x, 1e-7), _err(x, ref.x)
    else:
        xs = oprob.exact(o)
        assert _close(x, xs, 1e-7), _err(x, xs)


def test_served_96_mixed_full_size():
    _say("[gpu] served 96^3 / 48^3 / 20^3 hierarchy, 512 fine subdomains (mixed)")
    meshes = W.served_hierarchy(96)
    nps = [W.nparts_rule(m.nv) for m in meshes[:-1]]
    pb = W.Problem("served96", meshes, nps, W.kappa_draw(5003, 5004), precision="mixed")
    s, h, keep = _system(pb, "mixed")
    A, b = fem.assemble(meshes[0], pb.kappa)
    x, info = s.solve(b)
    _say(f"[gpu] 96^3 mixed: {info.iterations} iterations, relres {info.relres:.2e}")
    assert info.status == 0 and info.relres <= 1e-8
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    _check_smoother_samples(s, meshes[0], A, nps[0], [0, 73, 146, 219, 292, 365, 438, 511], 1e-2)


def test_batched_32_instances_full_size():
    """The batched workload as benchmarked (32 ragged instances, fine n in
    {24, 32, 40, 48, 64}, mixed precision, dense solves through inverse
    panels, one launch sequence per Arnoldi step): every slot reaches the
    true relative residual 1e-8 computed from the oracle's assembly of its
    own fine level, and equals its solve alone bit for bit."""
    nnms = _gpu()
    _say("[gpu] 32 batched instances (mixed)")
    probs = W.batched_instances(count=32)
    keep, systems, bs, As = [], [], [], []
    for pb in probs:
        ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
        h = nnms.Hierarchy(ms, pb.nparts, overlap=pb.overlap, its=pb.its, precision=nnms.MIXED,
                           dense_apply=nnms.INVERSE)
        s = nnms.System(h, pb.kappa, 1.0)
        keep.append((ms, h))
        systems.append(s)
        A, b = fem.assemble(pb.meshes[0], pb.kappa)
        As.append(A)
        bs.append(b)
    xs, infos = nnms.solve_batch(systems, bs)
    for i, (A, b, x, info) in enumerate(zip(As, bs, xs, infos)):
        assert info.status == 0 and info.relres <= 1e-8, i
        assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b), i
    for i in (0, 7, 31):
        x, info = systems[i].solve(bs[i])
        assert np.array_equal(x, xs[i]) and info.iterations == infos[i].iterations, i

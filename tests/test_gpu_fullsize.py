"""The default path (dense subdomain LU, barycentric transfer) at the
benchmark's full size and launch configuration (the tuned shapes of the
committed cache), against the FP64 oracle.

48^3 / 24^3 / 10^3, 64 + 8 subdomains: the assembled operators, the load
vector and both transfers on every entry (the same sums in another order,
1e-13 relative); the smoother on sampled subdomains, each solved by the
oracle one by one with LAPACK (its owned rows, 1e-9 relative: rounding
times the block's condition number); a full solve in FP64 against the
oracle's own FGMRES solution (same iteration count within one, 1e-7) and in
mixed precision against x* (1e-7; its FP32 smoother on sampled subdomains
to 1e-2, FP32 rounding times block condition numbers up to ~1e5).
96^3 / 48^3 / 20^3 (the largest served hierarchy, 512 fine subdomains,
mixed): the true residual of a solve computed from the oracle's assembly,
and sampled subdomains of the fine smoother.  The 32 batched instances:
true residuals and bitwise equality with solves alone.
"""
import os
import sys

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

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


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _system(pb, precision):
    nnms = _gpu()
    from paper_2412_08981_amd import autotune

    prec = nnms.MIXED if precision == "mixed" else nnms.FP64
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, overlap=pb.overlap, its=pb.its, precision=prec)
    s = nnms.System(h, pb.kappa, 1.0)
    autotune.tune(s, cache=CACHE)  # the benchmark's launch shapes
    s.destroy()
    return nnms.System(h, pb.kappa, 1.0), h, ms


def _check_smoother_samples(s, mesh, A, nparts, parts, tol):
    rng = np.random.default_rng(7)
    r = rng.standard_normal(mesh.nv)
    r[mesh.dirichlet != 0] = 0
    z = s.apply_smoother(0, r)
    owned, sets = schwarz.partition(mesh, nparts, 1)
    for p in parts:
        S = sets[p]
        y = sla.lu_solve(sla.lu_factor(A[S][:, S].toarray()), r[S])
        own = np.sort(owned[p])
        ref = y[np.searchsorted(S, own)]
        assert _rel(z[own], ref) <= tol, (p, _rel(z[own], ref))


def test_cube48_fp64_full_size():
    _say("[gpu] 48^3 / 24^3 / 10^3 at the benchmark's launch shapes (fp64)")
    pb = W.cube48_three_level("fp64")
    s, h, keep = _system(pb, "fp64")
    o = oprob.build(pb)
    for l in range(3):
        rp, col = h.csr(l)
        A = sp.csr_matrix((s.matrix_values(l), col, rp), shape=(s.n[l], s.n[l]))
        assert abs(A - o.A[l]).max() <= 1e-13 * abs(o.A[l]).max(), l
    assert np.abs(s.rhs() - o.b).max() <= 1e-14 * np.abs(o.b).max()
    rng = np.random.default_rng(3)
    for l in range(2):
        xc = rng.standard_normal(s.n[l + 1])
        assert _rel(s.apply_prolong(l, xc), o.P[l] @ xc) <= 1e-13
        x = rng.standard_normal(s.n[l])
        x[pb.meshes[l].dirichlet != 0] = 0
        assert _rel(s.apply_restrict(l, x), o.P[l].T @ x) <= 1e-13
        x = rng.standard_normal(s.n[l])
        x[pb.meshes[l].dirichlet != 0] = 0
        assert _rel(s.apply_operator(l, x), o.A[l] @ x) <= 1e-13
    _check_smoother_samples(s, pb.meshes[0], o.A[0], pb.nparts[0], [0, 21, 63], 1e-9)
    ref = oprob.solve(o)
    x, info = s.solve(o.b)
    _say(f"[gpu] 48^3 fp64: {info.iterations} iterations (oracle {ref.iterations})")
    assert info.status == 0 and info.relres <= 1e-8
    assert abs(info.iterations - ref.iterations) <= 1
    assert np.linalg.norm(o.b - o.A[0] @ x) <= 1e-8 * np.linalg.norm(o.b)
    assert _rel(x, ref.x) <= 1e-7


def test_cube48_mixed_full_size():
    _say("[gpu] 48^3 / 24^3 / 10^3 at the benchmark's launch shapes (mixed)")
    pb = W.cube48_three_level("mixed")
    s, h, keep = _system(pb, "mixed")
    A, b = fem.assemble(pb.meshes[0], pb.kappa)
    x, info = s.solve(b)
    assert info.status == 0 and info.relres <= 1e-8
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    xs = spla.splu(A.tocsc()).solve(b)  # x* by a sparse direct solve
    assert _rel(x, xs) <= 1e-7
    # FP32 smoother on sampled subdomains: FP32 rounding (6e-8) times the
    # block's condition number (up to ~1e5 with this kappa)
    _check_smoother_samples(s, pb.meshes[0], A, pb.nparts[0], [5, 40], 1e-2)


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
    _check_smoother_samples(s, meshes[0], A, nps[0], [0, 511], 1e-2)


def test_batched_32_instances_full_size():
    """The batched workload as benchmarked (32 ragged instances, fine n in
    {24, 32, 40, 48, 64}, mixed precision, one launch sequence per Arnoldi
    step): every slot reaches the true relative residual 1e-8 computed from
    the oracle's assembly of its own fine level, and equals its solve alone
    bit for bit."""
    nnms = _gpu()
    _say("[gpu] 32 batched instances (mixed)")
    probs = W.batched_instances(count=32)
    keep, systems, bs, As = [], [], [], []
    for pb in probs:
        ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
        h = nnms.Hierarchy(ms, pb.nparts, overlap=pb.overlap, its=pb.its, precision=nnms.MIXED)
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

"""Launch-shape autotuning: every candidate shape computes the same solve up
to rounding (the lanes per CSR row change the order of a row's partial sums;
the persistent grid changes nothing arithmetic), the chosen shapes are
stored in the hierarchy and reload from the cache."""
import json

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_keeps_results_and_caches(tmp_path):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08981_amd import autotune, nnms

    pb = W.Problem("t", W.make_hierarchy([14, 7, 3], [11, 12, 13]), [4, 2], W.kappa_draw(204, 205))
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts)
    s = nnms.System(h, pb.kappa)
    b = s.rhs()
    x0, i0 = s.solve(b)
    cache = str(tmp_path / "tuning.json")
    t = autotune.tune(s, cache=cache, reps=3)
    assert t["tuned"] == 1 and t["spmv_lanes"][0] in (0, 1, 4, 8, 16, 32, 64)
    assert t["pt_lanes"][0] in (0, 1, 2, 4, 8, 16, 32, 64)  # 2: P^T in column-sorted slices
    assert h.get_tuning() == t
    x1, i1 = s.solve(b)
    assert i1.iterations == i0.iterations and np.linalg.norm(x1 - x0) <= 1e-10 * np.linalg.norm(x0)
    x1b, _ = s.solve(b)
    assert np.array_equal(x1, x1b)  # a fixed shape is deterministic
    for g in (0, 1, 4, 8, 32, 64):  # 0, 1: sliced ELL layout (one or four waves per slice)
        d = dict(t)
        d["spmv_lanes"] = [g] * 8
        d["pt_lanes"] = [g] * 8
        d["krylov_lanes"] = g
        d["ras_groups"] = [256] * 8
        h.set_tuning(d)
        s2 = nnms.System(h, pb.kappa)
        x2, i2 = s2.solve(b)
        assert i2.status == 0 and abs(i2.iterations - i0.iterations) <= 1
        assert np.linalg.norm(x2 - x0) <= 1e-10 * np.linalg.norm(x0)
        s2.destroy()
    # cache round trip: a fresh hierarchy of the same shape takes the cached shapes without timing
    h2 = nnms.Hierarchy([nnms.Mesh.from_workload(m) for m in pb.meshes], pb.nparts)
    s3 = nnms.System(h2, pb.kappa)
    t3 = autotune.tune(s3, cache=cache)
    assert t3 == json.load(open(cache))[next(iter(json.load(open(cache))))]
    with pytest.raises(nnms.NNMSError):
        bad = dict(t)
        bad["spmv_lanes"] = [3] * 8
        h.set_tuning(bad)
    with pytest.raises(nnms.NNMSError):  # column-sorted slices exist for P^T only
        bad = dict(t)
        bad["spmv_lanes"] = [2] * 8
        h.set_tuning(bad)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_blocks_per_work_item_same_bits(precision):
    """Grouping K blocks per work item: K = 1 and K = 4 (blocks substituted
    one after the other) only change who computes a block, not the order of
    any sum, so their solves are bitwise identical; K = 2 applies the
    precomputed inverse of each 128 x 128 diagonal block pair (other
    rounding), so it agrees to rounding and is deterministic.  Every K
    matches the oracle's smoother on every level."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import problem as oprob
    from paper_2412_08981_amd import nnms

    pb = W.Problem("k", W.make_hierarchy([17, 8, 4], [21, 22, 23]), [4, 2], W.kappa_draw(204, 206),
                   precision=precision)
    prec = nnms.MIXED if precision == "mixed" else nnms.FP64
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, precision=prec)
    o = oprob.build(pb)
    base = h.get_tuning()
    ref = None
    rng = np.random.default_rng(5)
    for K in (1, 2, 4):
        d = dict(base)
        d["ras_blocks"] = [K] * 8
        h.set_tuning(d)
        s = nnms.System(h, pb.kappa)
        x, info = s.solve(o.b)
        assert info.status == 0 and info.relres <= 1e-8
        if ref is None:
            ref, ref_its = x, info.iterations
        elif K == 2:
            assert abs(info.iterations - ref_its) <= 1
            assert np.linalg.norm(x - ref) <= 1e-7 * np.linalg.norm(ref), K
            x2, _ = s.solve(o.b)
            assert np.array_equal(x, x2)
        else:
            assert np.array_equal(x, ref), K
        if precision == "fp64":
            for l in range(3):
                r = rng.standard_normal(s.n[l])
                r[pb.meshes[l].dirichlet != 0] = 0
                z = s.apply_smoother(l, r)
                zr = o.vcycle.levels[l].ras.apply(r) if l < 2 else np.linalg.solve(o.A[l].toarray(), r)
                assert np.linalg.norm(z - zr) <= 1e-9 * np.linalg.norm(zr), (K, l)
        s.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_of_differently_tuned_hierarchies_same_bits(precision):
    """Systems whose hierarchies carry different lanes-per-row choices (which
    fix the summation order; 0 and 1 = sliced ELL with one or four waves per
    slice) and different blocks per smoother work item (two-block items
    round differently) keep their own order inside one batch: every slot
    equals its solve alone, bitwise."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08981_amd import nnms

    prec = nnms.MIXED if precision == "mixed" else nnms.FP64
    keep, systems, bs, alone = [], [], [], []
    for n, g, gp, kb, seed in ((14, 4, 64, 1, 11), (12, 64, 8, 2, 21), (14, 0, 1, 4, 31), (13, 1, 0, 2, 41)):
        pb = W.Problem("t", W.make_hierarchy([n, n // 2, 3], [seed, seed + 1, seed + 2]), [4, 2],
                       W.kappa_draw(204, seed))
        ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
        h = nnms.Hierarchy(ms, pb.nparts, precision=prec)
        d = h.get_tuning()
        d["spmv_lanes"] = [g] * 8
        d["pt_lanes"] = [gp] * 8
        d["ras_blocks"] = [kb] * 8
        d["krylov_lanes"] = g
        h.set_tuning(d)
        s = nnms.System(h, pb.kappa)
        b = s.rhs()
        keep.append((ms, h))
        systems.append(s)
        bs.append(b)
        alone.append(s.solve(b))
    xs, infos = nnms.solve_batch(systems, bs)
    for k, (x, info) in enumerate(alone):
        assert infos[k].iterations == info.iterations
        assert np.array_equal(xs[k], x), k

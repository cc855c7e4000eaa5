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
    assert t["tuned"] == 1 and t["spmv_lanes"][0] in (4, 8, 16, 32, 64)
    assert h.get_tuning() == t
    x1, i1 = s.solve(b)
    assert i1.iterations == i0.iterations and np.linalg.norm(x1 - x0) <= 1e-10 * np.linalg.norm(x0)
    x1b, _ = s.solve(b)
    assert np.array_equal(x1, x1b)  # a fixed shape is deterministic
    for g in (4, 8, 32, 64):
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

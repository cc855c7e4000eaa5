"""Ragged batches through the C ABI: systems of different meshes, subdomain
counts and parameters solved in one launch sequence give the oracle's
solution and the same bits as when solved alone; the slot API (start / step
/ result) lets systems join a running batch."""
import numpy as np
import pytest

import workloads as W
from oracle import problem as oprob

pytestmark = pytest.mark.gpu


def _nnms():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08981_amd import nnms

    return nnms


def _problems(precision):
    out = []
    for i, (n, nps) in enumerate([(9, [2, 2]), (12, [4, 2]), (14, [8, 2]), (10, [2, 2])]):
        ns = W.coarse_sizes(n)
        meshes = W.make_hierarchy(ns, [700 + 10 * i + l for l in range(3)])
        out.append(W.Problem(f"b{i}", meshes, nps, W.kappa_draw(204, 709 + 10 * i), precision=precision))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ragged_batch_matches_alone_and_oracle(precision):
    nnms = _nnms()
    probs = _problems(precision)
    prec = nnms.MIXED if precision == "mixed" else nnms.FP64
    keep, systems, bs, xstar, oits = [], [], [], [], []
    for pb in probs:
        ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
        h = nnms.Hierarchy(ms, pb.nparts, precision=prec)
        s = nnms.System(h, pb.kappa)
        o = oprob.build(pb)
        keep.append((ms, h))
        systems.append(s)
        bs.append(o.b)
        xstar.append(oprob.exact(o))
        oits.append(oprob.solve(o).iterations)
    alone = [s.solve(b) for s, b in zip(systems, bs)]
    for graph in (True, False):
        xs, infos = nnms.solve_batch(systems, bs, graph=graph)
        for k in range(len(systems)):
            assert np.array_equal(xs[k], alone[k][0]), k
            assert infos[k].iterations == alone[k][1].iterations
            assert infos[k].status == 0 and infos[k].relres <= 1e-8
            assert np.linalg.norm(xs[k] - xstar[k]) <= 1e-7 * np.linalg.norm(xstar[k])
            tol = 1 if precision == "fp64" else max(1, int(0.1 * oits[k]) + 1)
            assert abs(infos[k].iterations - oits[k]) <= tol


def test_slots_join_a_running_batch():
    import torch

    nnms = _nnms()
    probs = _problems("mixed")[:3]
    keep, systems, bs = [], [], []
    for pb in probs:
        ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
        h = nnms.Hierarchy(ms, pb.nparts, precision=nnms.MIXED)
        s = nnms.System(h, pb.kappa)
        keep.append((ms, h))
        systems.append(s)
        bs.append(torch.from_numpy(s.rhs()).cuda())
    ref = [s.solve(b.cpu().numpy()) for s, b in zip(systems, bs)]
    # slot 0 starts alone; one step later slots 1 and 2 join (the batch is re-formed)
    b1 = nnms.Batch(systems[:1], graph=False)
    b1.start(0, bs[0].data_ptr())
    b1.step(1)
    b1.destroy()
    bt = nnms.Batch(systems, graph=True)
    bt.start(1, bs[1].data_ptr())
    bt.start(2, bs[2].data_ptr())
    while bt.step(1) > 0:
        pass
    for k in range(3):
        x = torch.zeros(systems[k].n[0], dtype=torch.float64, device="cuda")
        info = bt.result(k, x.data_ptr())
        torch.cuda.synchronize()
        assert info.status == 0 and info.iterations == ref[k][1].iterations
        assert np.array_equal(x.cpu().numpy(), ref[k][0])


def test_batch_start_and_result_follow_the_callers_stream():
    """nnms_batch_start reads b, and nnms_batch_result writes x, after the
    work already enqueued on the stream the batch was created with (here a
    long product and then the writes of b and x on a torch stream), and that
    stream's later work sees x."""
    import torch

    nnms = _nnms()
    pb = _problems("fp64")[1]
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts)
    s = nnms.System(h, pb.kappa)
    rhs = s.rhs()
    ref = s.solve(rhs)
    user = torch.cuda.Stream()
    big = torch.randn(4096, 4096, device="cuda", dtype=torch.float64)
    torch.cuda.synchronize()
    bt = nnms.Batch([s], stream=user)
    with torch.cuda.stream(user):
        t = big @ big  # keeps the caller's stream busy
        b = torch.zeros(s.n[0], dtype=torch.float64, device="cuda")
        b.copy_(torch.from_numpy(rhs).to("cuda", non_blocking=False))
    bt.start(0, b.data_ptr())
    while bt.step(1) > 0:
        pass
    with torch.cuda.stream(user):
        t = t @ big
        x = torch.full((s.n[0],), float("nan"), dtype=torch.float64, device="cuda")
    info = bt.result(0, x.data_ptr())
    with torch.cuda.stream(user):
        y = x * 1.0  # later work on the caller's stream
    user.synchronize()
    bt.destroy()
    assert info.status == 0 and info.iterations == ref[1].iterations
    assert np.array_equal(y.cpu().numpy(), ref[0])
    del t

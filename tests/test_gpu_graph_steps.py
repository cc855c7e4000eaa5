"""A solve enqueues as many Arnoldi steps as the plan's previous solve took
(replays of the plan's one-step HIP graph, back to back) before it reads
the running-slot count.  Steps after a
slot has converged leave it unchanged, so a solve's result and iteration
count do not depend on what the system solved before: after a longer solve
(more steps replayed than needed), after a shorter one (the graph ends
before convergence and single steps follow), and without graphs, every
result is bitwise the one of a fresh system."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08981_amd import nnms

    return nnms


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_independent_of_previous_step_count(precision):
    nnms = _gpu()
    prec = nnms.MIXED if precision == "mixed" else nnms.FP64
    pb = W.Problem("g", W.make_hierarchy([14, 7, 3], [111, 112, 113]), [4, 2], W.kappa_draw(204, 208))
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, precision=prec)
    b = nnms.System(h, pb.kappa).rhs()

    def fresh(rtol, graph=True):
        s = nnms.System(h, pb.kappa)
        out = s.solve(b, rtol=rtol, graph=graph)
        s.destroy()
        return out

    loose, tight = 1e-3, 1e-12
    xl, il = fresh(loose)
    xt, it = fresh(tight)
    assert il.status == 0 and it.status == 0 and it.iterations > il.iterations
    s = nnms.System(h, pb.kappa)
    for rtol, (xr, ir) in ((tight, (xt, it)), (loose, (xl, il)), (tight, (xt, it)), (tight, (xt, it))):
        x, info = s.solve(b, rtol=rtol)
        assert info.iterations == ir.iterations and info.status == 0, rtol
        assert np.array_equal(x, xr), rtol
    xn, inn = fresh(tight, graph=False)
    assert inn.iterations == it.iterations and np.array_equal(xn, xt)
    # a zero right-hand side after a solve: no steps change anything
    z, iz = s.solve(np.zeros_like(b))
    assert not np.any(z) and iz.iterations == 0
    x, info = s.solve(b, rtol=loose)
    assert info.iterations == il.iterations and np.array_equal(x, xl)
    s.destroy()

"""A hierarchy derived from one fine mesh by the coarsening of Algorithm 1
(Section 3.1) on the HIP path, against the FP64 oracle built on the
oracle's own coarsening of the same mesh (the two coarsenings are equal bit
for bit, checked on the CPU in test_host_setup.py and again here).

Tolerances as for the independently meshed hierarchies: solves reach
relres <= 1e-8 within one step of the oracle's iteration count and x* to
1e-7; one V-cycle application to 1e-9 relative."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import coarsen, problem as oprob

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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_coarsened_three_levels_match_oracle(precision):
    nnms = _gpu()
    _say(f"[gpu] coarsened hierarchy from a 14^3 mesh, 8 rounds per level ({precision})")
    fine = W.kuhn_cube(14, 31)
    # the library's levels
    m0 = nnms.Mesh.from_workload(fine)
    m1, _ = m0.coarsen(8, 1)
    m2, _ = m1.coarsen(8, 2)
    # the oracle's levels
    r1 = coarsen.coarsen(fine.xyz, fine.tets, fine.dirichlet, 8, 1)
    r2 = coarsen.coarsen(r1.xyz, r1.tets, r1.dirichlet, 8, 2)
    meshes = [fine, W.Mesh(r1.xyz, r1.tets.astype(np.int32), r1.dirichlet, 0),
              W.Mesh(r2.xyz, r2.tets.astype(np.int32), r2.dirichlet, 0)]
    for lib, ora in ((m1, r1), (m2, r2)):
        xyz, tets, d = lib.read()
        assert np.array_equal(xyz, ora.xyz) and np.array_equal(tets, ora.tets)
    pb = W.Problem("coarsened", meshes, [4, 2], W.kappa_draw(204, 205), precision=precision)
    prec = nnms.MIXED if precision == "mixed" else nnms.FP64
    h = nnms.Hierarchy([m0, m1, m2], pb.nparts, precision=prec)
    s = nnms.System(h, pb.kappa, 1.0)
    o = oprob.build(pb)
    if precision == "fp64":
        r = np.random.default_rng(41).standard_normal(s.n[0])
        r[fine.dirichlet != 0] = 0
        assert _rel(s.apply_vcycle(r), o.vcycle(r)) <= 1e-9
    ref = oprob.solve(o)
    x, info = s.solve(o.b)
    assert info.status == 0 and info.relres <= 1e-8
    if precision == "fp64":
        assert abs(info.iterations - ref.iterations) <= 1
    else:
        assert info.iterations <= int(np.ceil(1.1 * ref.iterations)) + 1
    assert _rel(x, oprob.exact(o)) <= 1e-7

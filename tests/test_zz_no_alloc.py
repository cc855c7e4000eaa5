"""nnms_apply_smoother_noalloc (the smoother for callers that cannot
allocate device memory, working in a per-GPU static scratch array) against
nnms_apply_smoother on the same system: bitwise equal on every level (dense
FP64, mixed precision, ILU, dense solves through inverse panels in both
precisions), two calls in a row with the second on a smaller system, and
tables beyond the scratch array's size refused."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08981_amd import nnms

    return nnms, torch


def _system(nnms, ns, seeds, nparts, **kw):
    meshes = [W.kuhn_cube(n, s) for n, s in zip(ns, seeds)]
    ms = [nnms.Mesh.from_workload(m) for m in meshes]
    h = nnms.Hierarchy(ms, nparts, **kw)
    return meshes, ms, h, nnms.System(h, W.kappa_draw(204, 205))


def _check(nnms, torch, meshes, s, level, seed):
    r = np.random.default_rng(seed).standard_normal(s.n[level])
    r[np.repeat(meshes[level].dirichlet, s.n[level] // meshes[level].nv) != 0] = 0
    ref = s.apply_smoother(level, r)
    rd = torch.from_numpy(r).cuda()
    zd = torch.full((s.n[level],), np.nan, dtype=torch.float64, device="cuda")
    s.apply_smoother_noalloc(level, rd.data_ptr(), zd.data_ptr())
    torch.cuda.synchronize()
    z = zd.cpu().numpy()
    assert np.array_equal(z, ref), (level, np.abs(z - ref).max())


@pytest.mark.parametrize("kind", ["fp64", "mixed", "ilu", "inverse", "inverse-mixed"])
def test_noalloc_equals_apply_smoother(env, kind):
    nnms, torch = env
    kw = {"precision": nnms.MIXED if kind.endswith("mixed") else nnms.FP64}
    if kind == "ilu":
        kw.update(subsolver=nnms.ILU, ilu_fill=[2, 0])
    if kind.startswith("inverse"):
        kw.update(dense_apply=nnms.INVERSE)
    big = _system(nnms, (13, 7, 4), (11, 12, 13), [8, 2], **kw)
    small = _system(nnms, (9, 5, 3), (21, 22, 23), [4, 2], **kw)
    # two calls in a row, the second on a smaller input, then every level
    _check(nnms, torch, big[0], big[3], 0, 1)
    _check(nnms, torch, small[0], small[3], 0, 2)
    for lvl in range(3):
        _check(nnms, torch, big[0], big[3], lvl, 3 + lvl)
        _check(nnms, torch, small[0], small[3], lvl, 7 + lvl)


def test_noalloc_refuses_oversized_tables(env):
    nnms, torch = env
    meshes, ms, h, s = _system(nnms, (27, 6), (31, 32), [16384])
    rd = torch.zeros(s.n[0], dtype=torch.float64, device="cuda")
    zd = torch.zeros(s.n[0], dtype=torch.float64, device="cuda")
    with pytest.raises(nnms.NNMSError) as e:
        s.apply_smoother_noalloc(0, rd.data_ptr(), zd.data_ptr())
    assert e.value.name == "INVALID_ARG"
    # the coarsest level still fits
    _check(nnms, torch, meshes, s, 1, 5)

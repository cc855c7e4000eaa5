"""Error paths of assemble(mesh, kappa) through the C ABI: a non-positive
kappa is refused before any device work (NNMS_ERR_INVALID_ARG), and a
factorisation whose pivots vanish reports NNMS_ERR_SINGULAR for the dense
and the ILU subdomain solvers alike.  The vanishing pivots come from a
kappa of 1e-320 (a subnormal) in mixed precision: the FP32 copies of the
subdomain matrices are exactly zero, so the first pivot is 0; nothing out
of bounds is touched and every kernel ends."""
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08981_amd import nnms

    return nnms


def _hier(nnms, **kw):
    pb = W.cube16_two_level()
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    return nnms.Hierarchy(ms, pb.nparts, **kw), ms


@pytest.mark.parametrize("value", [0.0, -1.0, float("nan")])
def test_nonpositive_kappa_is_refused(value):
    nnms = _gpu()
    h, keep = _hier(nnms)
    with pytest.raises(nnms.NNMSError) as e:
        nnms.System(h, W.KappaField("const", value), 1.0)
    assert e.value.name == "INVALID_ARG"
    # the hierarchy stays usable
    s = nnms.System(h, W.KappaField("const", 1.0), 1.0)
    x, info = s.solve(s.rhs())
    assert info.status == 0


@pytest.mark.parametrize("subsolver", ["lu", "ilu"])
def test_vanishing_pivots_are_singular(subsolver):
    nnms = _gpu()
    kw = {} if subsolver == "lu" else {"subsolver": nnms.ILU, "ilu_fill": [0]}
    h, keep = _hier(nnms, precision=nnms.MIXED, **kw)
    with pytest.raises(nnms.NNMSError) as e:
        nnms.System(h, W.KappaField("const", 1e-320), 1.0)
    assert e.value.name == "SINGULAR"

"""The library's host-side structure setup, called through the C ABI without a
GPU, against the oracle's independent implementations (no GPU)."""
import os
import re
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import coarsen, ilu, mls, schwarz, transfer

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

nnms = pytest.importorskip("paper_2412_08981_amd.nnms")


def _host(problem, overlap=1):
    ms = [nnms.Mesh.from_workload(m) for m in problem.meshes]
    h = nnms.Hierarchy(ms, problem.nparts, overlap=overlap, device=False)
    return ms, h


def test_header_symbols_are_exported():
    hdr = open(os.path.join(ROOT, "include", "nnms.h")).read()
    declared = set(re.findall(r"\b(nnms_[a-z_]+)\s*\(", hdr))
    out = subprocess.run(["nm", "-D", "--defined-only", nnms.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (nnms_[a-z_]+)", out))
    assert declared, "no declarations found"
    assert declared <= exported, declared - exported
    assert declared <= set(nnms.EXPORTED) | {"nnms_mesh_destroy"}


@pytest.mark.parametrize("cfg", ["cube16", "tiny3"])
def test_pattern_partition_transfer_match_oracle(cfg):
    if cfg == "cube16":
        pb = W.cube16_two_level()
    else:
        pb = W.Problem("tiny3", [W.kuhn_cube(9, 1), W.kuhn_cube(5, 2), W.kuhn_cube(3, 3)], [4, 2], W.KappaField())
    ms, h = _host(pb)
    for l, m in enumerate(pb.meshes):
        rp, col = h.csr(l)
        G = schwarz.vertex_graph(m.nv, m.tets).tocsr()
        for i in range(m.nv):
            row = col[rp[i]:rp[i + 1]]
            if m.dirichlet[i]:
                assert list(row) == [i]
            else:
                ref = G.indices[G.indptr[i]:G.indptr[i + 1]]
                ref = np.sort(ref[m.dirichlet[ref] == 0])
                assert np.array_equal(row, ref), i
        if l < len(pb.meshes) - 1:
            owned_o, sets_o = schwarz.partition(m, pb.nparts[l], pb.overlap)
            owner, sets = h.partition(l)
            assert len(sets) == len(sets_o)
            for p, (S, So) in enumerate(zip(sets, sets_o)):
                assert np.array_equal(S, So), p
                assert np.array_equal(np.nonzero(owner == p)[0], np.sort(owned_o[p]))
            idx, w = h.transfer(l)
            P_lib = np.zeros((m.nv, pb.meshes[l + 1].nv))
            for i in range(m.nv):
                for a in range(4):
                    P_lib[i, idx[i, a]] += w[i, a]
            P_or = transfer.interpolation(m, pb.meshes[l + 1]).toarray()
            assert np.abs(P_lib - P_or).max() <= 1e-14
        else:
            owner, sets = h.partition(l)
            assert len(sets) == 1 and np.array_equal(sets[0], np.nonzero(m.dirichlet == 0)[0])


def _csr_dense(rp, col, w, nr, nc):
    P = np.zeros((nr, nc))
    for i in range(nr):
        for e in range(rp[i], rp[i + 1]):
            P[i, col[e]] += w[e]
    return P


@pytest.mark.parametrize("alpha", [1.0, 1.5])
@pytest.mark.parametrize("cfg", ["cube16", "tiny3"])
def test_mls_transfer_matches_oracle(cfg, alpha):
    if cfg == "cube16":
        pb = W.cube16_two_level()
    else:
        pb = W.Problem("tiny3", [W.kuhn_cube(9, 1), W.kuhn_cube(5, 2), W.kuhn_cube(3, 3)], [4, 2], W.KappaField())
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, device=False, transfer=nnms.MLS, mls_alpha=alpha)
    for l in range(len(pb.meshes) - 1):
        f, c = pb.meshes[l], pb.meshes[l + 1]
        li = h.level_info(l)
        assert li.transfer == nnms.MLS
        rp, col, w = h.transfer_csr(l)
        P_or = mls.interpolation(f, c, alpha).tocsr()
        P_or.sort_indices()
        # same neighbourhoods (same scale decisions), values to rounding
        assert np.array_equal(rp, P_or.indptr)
        assert np.array_equal(col, P_or.indices)
        assert np.abs(w - P_or.data).max() <= 1e-12
        with pytest.raises(nnms.NNMSError):
            h.transfer(l)  # the four-entry form is barycentric only


def test_mls_restriction_matches_oracle():
    pb = W.Problem("tiny3", [W.kuhn_cube(9, 1), W.kuhn_cube(5, 2), W.kuhn_cube(3, 3)], [4, 2], W.KappaField())
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, device=False, transfer=nnms.MLS, mls_alpha=1.0, mls_restrict=True)
    for l in range(2):
        f, c = pb.meshes[l], pb.meshes[l + 1]
        li = h.level_info(l)
        assert li.mls_restrict == 1
        rp, col, w = h.restriction_csr(l)
        R = mls.restriction(f, c, 1.0).tocsr()
        R.sort_indices()
        assert np.array_equal(rp, R.indptr) and np.array_equal(col, R.indices)
        assert np.abs(w - R.data).max() <= 1e-11  # raw-basis oracle, fine-mesh scale
        # the prolongation is unchanged
        rpp, colp, wp = h.transfer_csr(l)
        P = mls.prolongation(f, c, 1.0).tocsr()
        P.sort_indices()
        assert np.array_equal(colp, P.indices) and np.abs(wp - P.data).max() <= 1e-12
    # without the option the restriction is the transpose of P
    h2 = nnms.Hierarchy(ms, pb.nparts, device=False, transfer=nnms.MLS, mls_alpha=1.0)
    rp, col, w = h2.restriction_csr(0)
    rpp, colp, wp = h2.transfer_csr(0)
    import scipy.sparse as sp
    PT = sp.csr_matrix((wp, colp, rpp), shape=(pb.meshes[0].nv, pb.meshes[1].nv)).T.tocsr()
    RT = sp.csr_matrix((w, col, rp), shape=PT.shape)
    assert abs(RT - PT).max() == 0


def test_barycentric_transfer_csr_matches_four_entry_form():
    pb = W.cube16_two_level()
    ms, h = _host(pb)
    f, c = pb.meshes
    rp, col, w = h.transfer_csr(0)
    idx, w4 = h.transfer(0)
    P4 = np.zeros((f.nv, c.nv))
    for i in range(f.nv):
        for a in range(4):
            P4[i, idx[i, a]] += w4[i, a]
    assert h.level_info(0).transfer == nnms.BARYCENTRIC
    assert np.array_equal(_csr_dense(rp, col, w, f.nv, c.nv), P4)
    assert np.all(c.dirichlet[col] == 0)


def test_mls_rejects_bad_scale():
    pb = W.cube16_two_level()
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    for a in (0.0, -1.0, float("nan")):
        with pytest.raises(nnms.NNMSError) as e:
            nnms.Hierarchy(ms, pb.nparts, device=False, transfer=nnms.MLS, mls_alpha=a)
        assert e.value.name == "INVALID_ARG"


@pytest.mark.parametrize("fill", [[0, 0], [1, 0], [2, 1]])
def test_ilu_patterns_match_oracle(fill):
    pb = W.Problem("tiny3", [W.kuhn_cube(9, 1), W.kuhn_cube(5, 2), W.kuhn_cube(3, 3)], [4, 2], W.KappaField())
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, device=False, subsolver=nnms.ILU, ilu_fill=fill)
    from oracle import fem
    for l in range(2):
        m = pb.meshes[l]
        A, _ = fem.assemble(m, pb.kappa)
        li = h.level_info(l)
        assert li.subsolver == nnms.ILU and li.ilu_nnz > 0
        rp, col = h.ilu_pattern(l)
        owner, sets = h.partition(l)
        row = 0
        for S in sets:
            cols, _ = ilu.symbolic(A[S][:, S].tocsr(), fill[l])
            for i in range(len(S)):
                assert np.array_equal(col[rp[row]:rp[row + 1]], cols[i]), (l, row)
                row += 1
        assert rp[row] == li.ilu_nnz
    assert h.level_info(2).subsolver == nnms.LU  # the coarsest level is solved directly


def test_ilu_rows_too_long_are_rejected():
    # a high fill level on a 9^3 subdomain fills rows far beyond what a
    # group of lanes can stage: a clear error at setup, not at launch
    pb = W.Problem("t", [W.kuhn_cube(9, 1), W.kuhn_cube(4, 2)], [1], W.KappaField())
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    with pytest.raises(nnms.NNMSError) as e:
        nnms.Hierarchy(ms, pb.nparts, device=False, subsolver=nnms.ILU, ilu_fill=[40])
    assert e.value.name == "INVALID_ARG" and "too long" in str(e.value)


def test_ilu_rejects_bad_fill():
    pb = W.cube16_two_level()
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    with pytest.raises(nnms.NNMSError) as e:
        nnms.Hierarchy(ms, pb.nparts, device=False, subsolver=nnms.ILU, ilu_fill=[-1])
    assert e.value.name == "INVALID_ARG"


@pytest.mark.parametrize("n,rounds,seed", [(7, 1, 3), (9, 8, 7), (12, 4, 19), (16, 8, 5)])
def test_coarsening_matches_oracle(n, rounds, seed):
    """Algorithm 1 in the library equals the oracle's, bit for bit (same
    MIS, same contraction choices, same output numbering)."""
    m = W.kuhn_cube(n, seed)
    r = coarsen.coarsen(m.xyz, m.tets, m.dirichlet, rounds, seed)
    c, removed = nnms.Mesh.from_workload(m).coarsen(rounds, seed)
    xyz, tets, d = c.read()
    assert removed == r.removed
    assert np.array_equal(xyz, r.xyz) and np.array_equal(tets, r.tets) and np.array_equal(d, r.dirichlet)
    # a coarsened mesh is a valid coarse level: point location of every
    # fine vertex succeeds and the hierarchy sets up
    h = nnms.Hierarchy([nnms.Mesh.from_workload(m), c], [2], device=False)
    assert h.level_info(1).nv == len(xyz)


@pytest.mark.parametrize("name", ["regular", "lopsided", "flat02", "flat007", "flat005"])
def test_coarsening_hand_checked_stars(name):
    """The library's contraction choice on the bipyramid stars whose
    qualities are closed forms (tests/golden/tet_quality.txt): the same
    elements as fixed by hand, and the vertex kept below the quality floor."""
    from test_oracle_coarsen import expected_star_tets, quality_golden

    rows, _ = quality_golden()
    hd, he, _, _, _, expected = rows[name]
    m = W.bipyramid_star(hd, he)
    c, removed = nnms.Mesh.from_workload(m).coarsen(1, 9)
    xyz, tets, d = c.read()
    if expected == "keep":
        assert removed == 0 and np.array_equal(tets, m.tets)
        return
    assert removed == 1 and np.array_equal(xyz, m.xyz[:5])
    assert {frozenset(int(x) for x in t) for t in tets} == expected_star_tets(expected)


def test_coarsening_rejects_bad_arguments():
    m = nnms.Mesh.from_workload(W.kuhn_cube(3, 1))
    with pytest.raises(nnms.NNMSError) as e:
        m.coarsen(-1, 0)
    assert e.value.name == "INVALID_ARG"


def test_level_info_counts():
    pb = W.cube16_two_level()
    ms, h = _host(pb)
    li = h.level_info(0)
    assert (li.nv, li.nt, li.nnz) == (4913, 24576, 46941)
    assert li.ninterior == 15 ** 3 and li.nparts == 8
    li1 = h.level_info(1)
    assert li1.nparts == 1 and li1.ninterior == 125 and li1.max_block == 125


def test_default_nparts_rule():
    pb = W.Problem("d", [W.kuhn_cube(24, 1), W.kuhn_cube(12, 2), W.kuhn_cube(5, 3)], [0, 0], W.KappaField())
    ms, h = _host(pb)
    assert h.level_info(0).nparts == 8  # 15625 vertices
    assert h.level_info(1).nparts == 2  # 2197 vertices
    assert W.nparts_rule(117649) == 64 and W.nparts_rule(912673) == 512


def test_bad_mesh_rejected():
    m = W.kuhn_cube(2, 1)
    tets = m.tets.copy()
    tets[3, [1, 2]] = tets[3, [2, 1]]  # inverted
    with pytest.raises(nnms.NNMSError) as e:
        nnms.Mesh(m.xyz, tets, m.dirichlet)
    assert e.value.name == "BAD_MESH"
    tets = m.tets.copy()
    tets[0, 0] = m.nv + 5
    with pytest.raises(nnms.NNMSError) as e:
        nnms.Mesh(m.xyz, tets, m.dirichlet)
    assert e.value.name == "BAD_MESH"


def test_point_location_error():
    f = W.kuhn_cube(4, 1)
    c = W.kuhn_cube(3, 2)
    xyz = c.xyz * 0.5  # coarse mesh covers only [0, 0.5]^3
    mf, mc = nnms.Mesh.from_workload(f), nnms.Mesh(xyz, c.tets, c.dirichlet)
    with pytest.raises(nnms.NNMSError) as e:
        nnms.Hierarchy([mf, mc], [2], device=False)
    assert e.value.name == "POINT_LOCATION"


def test_invalid_options():
    pb = W.cube16_two_level()
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    with pytest.raises(nnms.NNMSError) as e:
        nnms.Hierarchy(ms, [6], device=False)  # not a power of two
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(nnms.NNMSError):
        nnms.Hierarchy(ms, [8], its=0, device=False)


def test_dirichlet_default_is_bounding_box():
    m = W.kuhn_cube(3, 4)
    a = nnms.Mesh(m.xyz, m.tets, None)
    h = nnms.Hierarchy([a], [], device=False)
    owner, sets = h.partition(0)
    assert np.array_equal(owner >= 0, m.dirichlet == 0)


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the binding before PyTorch must not map a second HIP runtime
    (two runtimes in one process leave the later one without a device)."""
    code = ("import re, sys; sys.path.insert(0, %r)\n"
            "from paper_2412_08981_amd import nnms\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read()\n"
            "print(len(set(re.findall(r'(\\S*libamdhip64\\S*)', maps))))\n") % ROOT
    out = subprocess.run(["python", "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"


def test_field_split_structure_matches_oracle():
    """Three unknowns per vertex (linear elasticity, field splitting): the
    library's pattern equals the oracle's elasticity matrix pattern, its
    subdomains are the vertex subdomains carried to every component, and its
    transfer equals the oracle's split interpolation sum_f R_f^T P R~_f."""
    from oracle import elasticity as el

    pb = W.Problem("el", [W.kuhn_cube(7, 41), W.kuhn_cube(4, 42), W.kuhn_cube(3, 43)], [4, 2],
                   W.kappa_draw(204, 205))
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, device=False, ncomp=3)
    for l, m in enumerate(pb.meshes):
        li = h.level_info(l)
        assert (li.nv, li.ncomp, li.ndof) == (m.nv, 3, 3 * m.nv)
        assert li.ninterior == int((m.dirichlet == 0).sum())
        A, _ = el.assemble(m, pb.kappa, 0.3)
        rp, col = h.csr(l)
        assert np.array_equal(rp, A.indptr) and np.array_equal(col, A.indices)
        if l + 1 < len(pb.meshes):
            owner, sets = h.partition(l)
            _, sets_o = el.expand_sets(*schwarz.partition(m, pb.nparts[l], pb.overlap))
            assert len(sets) == len(sets_o) and all(np.array_equal(a, b) for a, b in zip(sets, sets_o))
            P = el.split_interpolation(transfer.interpolation(m, pb.meshes[l + 1]))
            prp, pcol, pw = h.transfer_csr(l)
            Pl = sp.csr_matrix((pw, pcol, prp), shape=P.shape)
            assert abs(Pl - P).max() <= 1e-14
            rrp, rcol, rw = h.restriction_csr(l)
            R = sp.csr_matrix((rw, rcol, rrp), shape=P.T.shape)
            assert abs(R - P.T).max() <= 1e-14


def test_field_split_default_subdomains_count_unknowns():
    pb = W.cube16_two_level()
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, [0], device=False, ncomp=3)
    assert h.level_info(0).nparts == W.nparts_rule(3 * pb.meshes[0].nv)


@pytest.mark.parametrize("restrict", [False, True])
def test_clipped_mls_matches_oracle(restrict):
    """MLS neighbourhoods clipped to the overlapping subdomain of the target's
    processor (both levels split across the fine level's subdomain count):
    the library's operators have the oracle's neighbourhoods and entries."""
    pb = W.Problem("tiny3", [W.kuhn_cube(9, 1), W.kuhn_cube(5, 2), W.kuhn_cube(3, 3)], [4, 2], W.KappaField())
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    h = nnms.Hierarchy(ms, pb.nparts, device=False, transfer=nnms.MLS, mls_alpha=1.0, mls_clip=True,
                       mls_restrict=restrict)
    hu = nnms.Hierarchy(ms, pb.nparts, device=False, transfer=nnms.MLS, mls_alpha=1.0, mls_restrict=restrict)
    for l in range(2):
        f, c = pb.meshes[l], pb.meshes[l + 1]
        rp, col, w = h.transfer_csr(l)
        P = mls.prolongation(f, c, 1.0, clip_parts=pb.nparts[l]).tocsr()
        P.sort_indices()
        assert np.array_equal(rp, P.indptr) and np.array_equal(col, P.indices)
        assert np.abs(w - P.data).max() <= 1e-12
        urp, ucol, uw = hu.transfer_csr(l)
        Pu = sp.csr_matrix((uw, ucol, urp), shape=P.shape)
        assert abs(P - Pu).max() > 1e-6  # clipping changes some rows
        if restrict:
            rp, col, w = h.restriction_csr(l)
            R = mls.restriction(f, c, 1.0, clip_parts=pb.nparts[l]).tocsr()
            R.sort_indices()
            assert np.array_equal(rp, R.indptr) and np.array_equal(col, R.indices)
            assert np.abs(w - R.data).max() <= 1e-11


def test_dense_apply_option():
    """The inverse-panel option is reported per dense level (the coarsest
    level too, ILU levels never), costs more device memory per system than
    the sweeps (the packed panels and their partial sums beside the LU), and
    an unknown value is refused."""
    pb = W.Problem("t3", [W.kuhn_cube(9, 1), W.kuhn_cube(5, 2), W.kuhn_cube(3, 3)], [4, 2], W.KappaField())
    ms = [nnms.Mesh.from_workload(m) for m in pb.meshes]
    hs = nnms.Hierarchy(ms, pb.nparts, device=False)
    hi = nnms.Hierarchy(ms, pb.nparts, device=False, dense_apply=nnms.INVERSE)
    assert all(hs.level_info(l).dense_apply == nnms.SWEEPS for l in range(3))
    assert all(hi.level_info(l).dense_apply == nnms.INVERSE for l in range(3))
    assert hi.system_bytes() > hs.system_bytes()
    hl = nnms.Hierarchy(ms, pb.nparts, device=False, subsolver=nnms.ILU, dense_apply=nnms.INVERSE)
    assert [hl.level_info(l).dense_apply for l in range(3)] == [nnms.SWEEPS, nnms.SWEEPS, nnms.INVERSE]
    with pytest.raises(nnms.NNMSError) as e:
        nnms.Hierarchy(ms, pb.nparts, device=False, dense_apply=7)
    assert e.value.name == "INVALID_ARG"

"""C ABI checks that need no GPU: the library loads, exports every entry
point declared in include/gdsw.h, and its host symbolic analysis (phase (a))
reproduces the oracle's integer maps bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2304_04876_amd import binding as B
from paper_2304_04876_amd import problems as P
from oracle import gdsw_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gdsw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gdsw_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared()
    assert "gdsw_setup" in names and "gdsw_apply" in names and "gdsw_solve" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(B.EXPORTED) == set(names)


def test_status_strings_and_defaults():
    assert B.gdsw_status_string(0) == "ok"
    assert "singular" in B.gdsw_status_string(2)
    o = B.gdsw_default_options()
    assert (o.overlap, o.coarse, o.local, o.jacobi_sweeps, o.local_prec) == (1, 1, 0, 5, 0)


def _maps_equal(pr, Z=None, overlap=1, local="exact", coarse="gdsw", sharing=None):
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, pr.dpn, Z,
                       B.gdsw_default_options(overlap=overlap, local=0 if local == "exact" else 1,
                                              coarse=B.COARSE_RGDSW if coarse == "rgdsw" else B.COARSE_GDSW),
                       sharing=sharing)
    try:
        M = O.GDSW(pr.A, pr.part, pr.dpn, pr.n_parts, Z=Z, overlap=overlap, local=local, coarse_space=coarse,
                   sharing=sharing)
        m = M.maps()
        ov_ptr = np.concatenate([[0], np.cumsum([r.size for r in M.R])])
        assert np.array_equal(B.gdsw_copy_map(h, B.MAP_OV_PTR), ov_ptr)
        assert np.array_equal(B.gdsw_copy_map(h, B.MAP_OV_IDX), m["ov_idx"])
        assert np.array_equal(B.gdsw_copy_map(h, B.MAP_IS_GAMMA), m["is_gamma"])
        assert np.array_equal(B.gdsw_copy_map(h, B.MAP_COMP_OF_NODE), m["comp_of_node"])
        assert np.array_equal(B.gdsw_copy_map(h, B.MAP_COMP_RANK), m["comp_rank"])
        info = B.gdsw_get_info(h)
        assert info["n0"] == m["n0"] and info["n_components"] == m["n_comp"]
        # Phi's column pattern: every interface dof in its component's columns
        rp = B.gdsw_copy_map(h, B.MAP_PHI_ROWPTR)
        cols = B.gdsw_copy_map(h, B.MAP_PHI_COL)
        phi = M.cs.phi.tocsr() if M.cs is not None else None
        if phi is not None:
            for d in np.linspace(0, pr.n - 1, 50).astype(int):
                lib_cols = set(cols[rp[d]:rp[d + 1]].tolist())
                or_cols = set(phi.indices[phi.indptr[d]:phi.indptr[d + 1]].tolist())
                assert or_cols <= lib_cols
    finally:
        B.gdsw_destroy(h)


@pytest.mark.parametrize("N,Pn", [(20, 2), (12, 3), (17, 3), (9, 2)])
def test_maps_poisson(N, Pn):
    _maps_equal(P.poisson3d(N, Pn))


@pytest.mark.parametrize("overlap", [0, 2])
def test_maps_overlap(overlap):
    _maps_equal(P.poisson3d(12, 3), overlap=overlap)


def test_maps_uneven_partition():
    pr = P.poisson3d(10, (2, 3, 1))
    _maps_equal(pr)


def test_maps_elasticity():
    pr = P.elasticity_q1(6, 2)
    _maps_equal(pr, P.rigid_body_modes(pr))


def test_maps_elasticity_three_boxes():
    pr = P.elasticity_q1(9, 3)
    _maps_equal(pr, P.rigid_body_modes(pr))


def test_maps_diffusion():
    spec = P.batch_diffusion_specs(3)[1]
    _maps_equal(P.batch_diffusion_problem(spec))


@pytest.mark.parametrize("case", ["poisson20", "poisson12", "elasticity6", "elasticity9", "diffusion"])
def test_maps_reduced_coarse_space(case):
    """Reduced GDSW: the coarse dimension, the columns touching each
    component and Phi's column pattern equal the oracle's."""
    if case == "poisson20":
        _maps_equal(P.poisson3d(20, 2), coarse="rgdsw")
    elif case == "poisson12":
        _maps_equal(P.poisson3d(12, 3), coarse="rgdsw")
    elif case.startswith("elasticity"):
        pr = P.elasticity_q1(int(case[10:]), 2 if case == "elasticity6" else 3)
        _maps_equal(pr, P.rigid_body_modes(pr), coarse="rgdsw")
    else:
        _maps_equal(P.batch_diffusion_problem(P.batch_diffusion_specs(3)[1]), coarse="rgdsw")


def test_closed_form_counts_small_workload():
    pr = P.workload_poisson_small()
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1)
    info = B.gdsw_get_info(h)
    B.gdsw_destroy(h)
    assert (info["n_gamma_nodes"], info["n_components"], info["sum_overlap_dofs"]) == (1141, 19, 10400)


@pytest.mark.slow
def test_closed_form_counts_large_workload():
    pr = P.workload_poisson_large()
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1, options=B.gdsw_default_options(local=1))
    info = B.gdsw_get_info(h)
    B.gdsw_destroy(h)
    assert (info["n_gamma_nodes"], info["n_components"], info["sum_overlap_dofs"]) == (325591, 2863, 2785280)


def test_invalid_arguments_are_reported():
    pr = P.poisson3d(6, 2)
    bad = pr.part.copy()
    bad[0] = 99
    with pytest.raises(B.GdswError) as e:
        B.gdsw_analyze(pr.A, bad, pr.n_parts, 1)
    assert e.value.status == 1 and "part" in str(e.value)
    A = pr.A.tolil()
    A[0, 1] = -2.0          # breaks symmetry
    with pytest.raises(B.GdswError) as e:
        B.gdsw_analyze(A.tocsr(), pr.part, pr.n_parts, 1)
    assert "symmetric" in str(e.value)
    with pytest.raises(B.GdswError):
        B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1, options=B.gdsw_default_options(jacobi_sweeps=0))
    A = pr.A.tolil()
    A[3, 3] = np.nan
    with pytest.raises(B.GdswError):
        B.gdsw_analyze(A.tocsr(), pr.part, pr.n_parts, 1)


def test_factor_without_analysis_state_error():
    # a handle whose analysis failed cannot be factored
    pr = P.poisson3d(6, 2)
    h = B.ctypes.c_void_p()
    rowptr, col, val = B._csr_arrays(pr.A)
    csr = B.CSR(pr.n, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data)
    bad = np.full(pr.n, 7, dtype=np.int32)
    st = B.lib().gdsw_analyze(B.ctypes.byref(csr), bad.ctypes.data, 2, 1, None, 0, None, B.ctypes.byref(h))
    assert st == 1
    assert "part" in B.gdsw_last_error(h.value)
    assert B.lib().gdsw_factor(h.value, None) == 7
    B.gdsw_destroy(h.value)


def test_set_launch_before_factor_state_error():
    pr = P.poisson3d(6, 2)
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1)
    assert B.lib().gdsw_set_launch(h, 0, 0, 1, 0, None) == 7
    assert "factor" in B.gdsw_last_error(h)
    assert B.lib().gdsw_set_launch(None, 0, 0, 1, 0, None) == 1
    B.gdsw_destroy(h)


def test_profile_before_factor_state_error():
    pr = P.poisson3d(6, 2)
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1)
    assert B.lib().gdsw_profile_local(h, 1) == 7
    assert "factor" in B.gdsw_last_error(h)
    count = ctypes.c_int32(-1)
    assert B.lib().gdsw_profile_read(h, None, 0, ctypes.byref(count)) == 7
    assert B.lib().gdsw_profile_read(h, None, 4, ctypes.byref(count)) == 1   # ms missing
    assert B.lib().gdsw_profile_read(h, None, 0, None) == 1                  # count missing
    assert B.lib().gdsw_profile_local(None, 1) == 1
    B.gdsw_destroy(h)


def test_profile_max_matches_header():
    text = open(os.path.join(ROOT, "include", "gdsw.h")).read()
    m = re.search(r"#define GDSW_PROFILE_MAX (\d+)", text)
    assert m and int(m.group(1)) == B.PROFILE_MAX


@pytest.mark.parametrize("level", [0, 1, 2])
@pytest.mark.parametrize("case", ["poisson", "diffusion", "elasticity"])
def test_iluk_patterns_match_oracle(level, case):
    """The library's ILU(k) patterns of every local matrix equal the oracle's
    level-of-fill patterns (an independent implementation of the same rule)."""
    if case == "poisson":
        pr = P.poisson3d(9, 2)
    elif case == "diffusion":
        rng = np.random.default_rng(1)
        pr = P.diffusion3d(8, np.exp(rng.standard_normal(9 ** 3)), 2)
    else:
        pr = P.elasticity_q1(4, 2)
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, pr.dpn, None,
                       B.gdsw_default_options(local=B.LOCAL_ILU0, ilu_level=level))
    rp = B.gdsw_copy_map(h, B.MAP_LOCAL_ROWPTR)
    cols = B.gdsw_copy_map(h, B.MAP_LOCAL_COL)
    ovp = B.gdsw_copy_map(h, B.MAP_OV_PTR)
    ovi = B.gdsw_copy_map(h, B.MAP_OV_IDX)
    B.gdsw_destroy(h)
    for i in range(pr.n_parts):
        d = ovi[ovp[i]:ovp[i + 1]]
        Ai = pr.A[d][:, d].tocsr()
        Pm, _ = O.iluk_pattern(Ai, level)
        r = rp[ovp[i]:ovp[i + 1] + 1]
        assert np.array_equal(r - r[0], Pm.indptr), i
        assert np.array_equal(cols[r[0]:r[-1]], Pm.indices), i


def test_ilu_options_validated():
    pr = P.poisson3d(6, 2)
    for bad in (dict(ilu_level=-1), dict(ilu_level=9), dict(ilu_factor_sweeps=-2)):
        with pytest.raises(B.GdswError):
            B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1, None,
                           B.gdsw_default_options(local=B.LOCAL_ILU0, **bad))


def test_size_limits_and_degenerate_inputs():
    """Limits and degenerate inputs are refused with INVALID_ARG, not run:
    an empty matrix; an ILU subdomain beyond the 16-bit local column range
    (41^3 = 68,921 dofs in one subdomain); a partition with an empty
    subdomain is accepted (the empty subdomain has no rows)."""
    import scipy.sparse as sp
    empty = sp.csr_matrix((0, 0))
    with pytest.raises(B.GdswError) as e:
        B.gdsw_analyze(empty, np.zeros(0, dtype=np.int32), 1, 1)
    assert e.value.status == 1
    pr = P.poisson3d(41, 1)
    with pytest.raises(B.GdswError) as e:
        B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1, options=B.gdsw_default_options(local=B.LOCAL_ILU0))
    assert e.value.status == 1 and "65535" in str(e.value)
    # the same subdomain is fine for the exact (band) local solver
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1)
    assert B.gdsw_get_info(h)["max_local_rows"] == 41 ** 3
    B.gdsw_destroy(h)
    # three parts named, the last one empty
    pr = P.poisson3d(8, 2)
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts + 1, 1)
    info = B.gdsw_get_info(h)
    ovp = B.gdsw_copy_map(h, B.MAP_OV_PTR)
    assert info["n_parts"] == pr.n_parts + 1 and ovp[-1] == ovp[-2]
    B.gdsw_destroy(h)


@pytest.mark.parametrize("Ne,Pn,coarse", [(6, 2, "gdsw"), (9, 3, "gdsw"), (9, 3, "rgdsw")])
def test_maps_element_sharing(Ne, Pn, coarse):
    """The interface from the element decomposition's sharing sets
    (gdsw_analyze_sharing): maps equal the oracle's bit for bit."""
    pr = P.elasticity_q1(Ne, Pn)
    _maps_equal(pr, Z=P.rigid_body_modes(pr), coarse=coarse, sharing=P.element_sharing(pr))


def test_sharing_sets_rejected_when_inconsistent():
    pr = P.elasticity_q1(6, 2)
    Z = P.rigid_body_modes(pr)
    ptr, sub = P.element_sharing(pr)
    # every node alone in its own subdomain: interior nodes then touch other subdomains
    own = (np.arange(pr.n_nodes + 1, dtype=np.int64), pr.part.astype(np.int32))
    with pytest.raises(B.GdswError) as e:
        B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 3, Z, sharing=own)
    assert e.value.status == 1 and "interior node" in str(e.value)
    # a set without the node's own subdomain
    bad = sub.copy()
    v = int(np.argmax(np.diff(ptr) == 1))
    bad[ptr[v]] = (pr.part[v] + 1) % pr.n_parts
    with pytest.raises(B.GdswError) as e:
        B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 3, Z, sharing=(ptr, bad))
    assert e.value.status == 1 and "own subdomain" in str(e.value)
    # an id out of range
    bad = sub.copy()
    bad[0] = pr.n_parts
    with pytest.raises(B.GdswError):
        B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 3, Z, sharing=(ptr, bad))


def test_element_sharing_full_size_counts():
    """The 48^3 Q1 elasticity mesh in 6^3 boxes: the element sharing sets give
    the geometric faces, edges and vertices (n_c = 540 + 450 + 125 = 1,115,
    n_0 = 6*540 + 5*450 + 3*125 = 5,865; the node-graph interface of R6 gives
    1,940 / 9,240)."""
    pr = P.elasticity_q1(48, 6)
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 3, P.rigid_body_modes(pr), sharing=P.element_sharing(pr))
    try:
        info = B.gdsw_get_info(h)
        assert (info["n_components"], info["n0"]) == (1115, 5865)
    finally:
        B.gdsw_destroy(h)

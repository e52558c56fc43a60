"""The nested-dissection supernodal structure of the exact local factor
(host analysis, no GPU): the maps it exports drive, in plain numpy here, the
same left-looking supernodal Cholesky and level-scheduled triangular solves
that the device kernels run; the factor must reproduce A_i = L L^T in the
new numbering and the solves must give A_i^{-1} r.  Also the structural
claims: the new numbering is a permutation per subdomain, every struct row
lies after its supernode, the rows by height cover each subdomain once, and
the factor holds fewer entries than the natural-order band."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2304_04876_amd import binding as B
from paper_2304_04876_amd import problems as P


def _maps(h):
    g = lambda m: B.gdsw_copy_map(h, m)   # noqa: E731
    sn = g(B.MAP_ND_SN).reshape(-1, 4)
    return dict(perm=g(B.MAP_ND_PERM), sn_ptr=g(B.MAP_ND_SN_PTR), first=sn[:, 0], ncol=sn[:, 1], nrow=sn[:, 2],
                height=sn[:, 3], voff=g(B.MAP_ND_VOFF), st_ptr=g(B.MAP_ND_ST_PTR), st_row=g(B.MAP_ND_ST_ROW),
                rc_ptr=g(B.MAP_ND_RC_PTR), rc=g(B.MAP_ND_RC).reshape(-1, 2), lv_base=g(B.MAP_ND_LV_BASE),
                lv_ptr=g(B.MAP_ND_LV_PTR), lv_rows=g(B.MAP_ND_LV_ROWS), up_ptr=g(B.MAP_ND_UP_PTR),
                up=g(B.MAP_ND_UP).reshape(-1, 4), rel=g(B.MAP_ND_REL), asm=g(B.MAP_ND_ASM).reshape(-1, 2),
                ov_ptr=g(B.MAP_OV_PTR), ov_idx=g(B.MAP_OV_IDX), rc_w=g(B.MAP_ND_RC_W), st_sn=g(B.MAP_ND_ST_SN),
                lv_info=g(B.MAP_ND_LV_INFO).reshape(-1, 4), ch_base=g(B.MAP_ND_CH_BASE),
                ch_row=g(B.MAP_ND_CH_ROW))


def _factor(m, Aval):
    """Left-looking supernodal Cholesky over the panels, as the device does."""
    L = np.zeros(int(m["voff"][-1]))
    L[m["asm"][:, 1]] = Aval[m["asm"][:, 0]]
    nsn = len(m["first"])
    for J in range(nsn):
        oJ, nJ, ldJ = m["voff"][J], m["ncol"][J], m["nrow"][J]
        PJ = L[oJ:oJ + ldJ * nJ].reshape(nJ, ldJ)   # [column, panel row]
        for u in range(m["up_ptr"][J], m["up_ptr"][J + 1]):
            K, s0, n1, ro = m["up"][u]
            oK, nK, ldK = m["voff"][K], m["ncol"][K], m["nrow"][K]
            PK = L[oK:oK + ldK * nK].reshape(nK, ldK)
            n2 = (m["st_ptr"][K + 1] - m["st_ptr"][K]) - s0
            rel = m["rel"][ro:ro + n2]
            rows = PK[:, nK + s0:nK + s0 + n2]            # (nK, n2)
            upd = rows.T @ rows[:, :n1]                   # (n2, n1)
            for b in range(n1):
                keep = rel >= rel[b]
                PJ[rel[b], rel[keep]] -= upd[keep, b]
        for j in range(nJ):
            d = PJ[j, j]
            assert d > 0
            PJ[j, j] = np.sqrt(d)
            PJ[j, j + 1:] /= PJ[j, j]
            for c in range(j + 1, nJ):
                PJ[c, c:] -= PJ[j, c] * PJ[j, c:]
    return L


def _check_subdomain(m, i, L, Ai_new, rng):
    n = Ai_new.shape[0]
    s0, s1 = m["sn_ptr"][i], m["sn_ptr"][i + 1]
    o = m["ov_ptr"][i]
    # L in the new numbering
    Ld = np.zeros((n, n))
    for J in range(s0, s1):
        f, nJ, ldJ = m["first"][J], m["ncol"][J], m["nrow"][J]
        PJ = L[m["voff"][J]:m["voff"][J] + ldJ * nJ].reshape(nJ, ldJ)
        st = m["st_row"][m["st_ptr"][J]:m["st_ptr"][J + 1]]
        assert len(st) == ldJ - nJ and (len(st) == 0 or st.min() >= f + nJ)
        rows = np.concatenate([np.arange(f, f + nJ), st])
        for c in range(nJ):
            Ld[rows[c:], f + c] = PJ[c, c:]
    A = Ai_new.toarray()
    assert np.abs(Ld @ Ld.T - A).max() <= 1e-12 * np.abs(A).max()
    # level-scheduled solves
    r = rng.uniform(-1, 1, n)
    y = r.copy()
    lb = m["lv_base"][i]
    nlev = m["lv_base"][i + 1] - lb - 1
    lptr = m["lv_ptr"][lb:lb + nlev + 1]
    lrows = m["lv_rows"][o:o + n]
    assert sorted(lrows.tolist()) == list(range(n))
    row_sn = np.empty(n, dtype=np.int64)
    for J in range(s0, s1):
        row_sn[m["first"][J]:m["first"][J] + m["ncol"][J]] = J

    def panel(J):
        nJ, ldJ = m["ncol"][J], m["nrow"][J]
        return L[m["voff"][J]:m["voff"][J] + ldJ * nJ].reshape(nJ, ldJ)

    for lev in range(nlev):
        rows = lrows[lptr[lev]:lptr[lev + 1]]
        t = {}
        for rr in rows:
            acc = y[rr]
            for q in range(m["rc_ptr"][o + rr], m["rc_ptr"][o + rr + 1]):
                K, pos = m["rc"][q]
                PK = panel(K)
                acc -= PK[:, pos] @ y[m["first"][K]:m["first"][K] + m["ncol"][K]]
            t[rr] = acc
        for J in sorted(set(row_sn[rows].tolist())):
            f, nJ = m["first"][J], m["ncol"][J]
            Ljj = panel(J)[:, :nJ].T                     # lower triangle, [row, column]
            y[f:f + nJ] = np.linalg.solve(np.tril(Ljj), np.array([t[f + c] for c in range(nJ)]))
    for lev in reversed(range(nlev)):
        rows = lrows[lptr[lev]:lptr[lev + 1]]
        for J in sorted(set(row_sn[rows].tolist())):
            f, nJ = m["first"][J], m["ncol"][J]
            PJ = panel(J)
            st = m["st_row"][m["st_ptr"][J]:m["st_ptr"][J + 1]]
            tJ = y[f:f + nJ] - PJ[:, nJ:] @ y[st]
            y[f:f + nJ] = np.linalg.solve(np.tril(PJ[:, :nJ].T).T, tJ)
    x = np.linalg.solve(A, r)
    assert np.abs(y - x).max() <= 1e-10 * np.abs(x).max()
    yd = _solve_by_passes(m, i, L, r)
    assert np.abs(yd - x).max() <= 1e-10 * np.abs(x).max()
    return np.count_nonzero(np.tril(Ld))


def _solve_by_passes(m, i, L, r):
    """The device's order of work: per height the gathers of the kept struct
    products (w), the inverted diagonal blocks, then the struct products of
    the height's supernodes into w; backward the struct parts against the
    final rows and the transposed inverted diagonal blocks."""
    s0, s1 = m["sn_ptr"][i], m["sn_ptr"][i + 1]
    o = m["ov_ptr"][i]
    sb = m["st_ptr"][s0]
    lb = m["lv_base"][i]
    nlev = m["lv_base"][i + 1] - lb - 1
    lp, info = m["lv_ptr"][lb:lb + nlev + 1], m["lv_info"][lb:lb + nlev + 1]
    n = len(r)

    def panel(J):
        nJ, ldJ = m["ncol"][J], m["nrow"][J]
        return L[m["voff"][J]:m["voff"][J] + ldJ * nJ].reshape(nJ, ldJ)

    inv = {J: np.linalg.inv(np.tril(panel(J)[:, :m["ncol"][J]].T)) for J in range(s0, s1)}
    row_sn = np.empty(n, dtype=np.int64)
    for J in range(s0, s1):
        row_sn[m["first"][J]:m["first"][J] + m["ncol"][J]] = J
    w = np.full(m["st_ptr"][s1] - sb, np.nan)
    y = r.astype(np.float64).copy()
    t = np.empty(n)
    for lev in range(nlev):
        rows = range(lp[lev], lp[lev + 1])
        for rr in rows:
            e0, e1 = m["rc_ptr"][o + rr], m["rc_ptr"][o + rr + 1]
            t[rr] = y[rr] - w[m["rc_w"][e0:e1]].sum()
        for rr in rows:
            J = row_sn[rr]
            f = m["first"][J]
            y[rr] = inv[J][rr - f, :rr - f + 1] @ t[f:rr + 1]
        for q in range(info[lev, 0], info[lev + 1, 0]):
            K = m["st_sn"][sb + q]
            fK, nK = m["first"][K], m["ncol"][K]
            w[q] = panel(K)[:, nK + (sb + q - m["st_ptr"][K])] @ y[fK:fK + nK]
    for lev in reversed(range(nlev)):
        rows = range(lp[lev], lp[lev + 1])
        for rr in rows:
            J = row_sn[rr]
            f, nJ = m["first"][J], m["ncol"][J]
            st = m["st_row"][m["st_ptr"][J]:m["st_ptr"][J + 1]]
            t[rr] = y[rr] - panel(J)[rr - f, nJ:] @ y[st]
        for rr in rows:
            J = row_sn[rr]
            f, nJ = m["first"][J], m["ncol"][J]
            c = rr - f
            y[rr] = inv[J][c:, c] @ t[f + c:f + nJ]
    return y


def _check_levels(m, i):
    """Supernodes numbered by height; per height the rows, the supernodes and
    their struct entries are consecutive; the multiply-add counts."""
    s0, s1 = m["sn_ptr"][i], m["sn_ptr"][i + 1]
    ht = m["height"][s0:s1]
    assert np.all(np.diff(ht) >= 0)
    o = m["ov_ptr"][i]
    n = m["ov_ptr"][i + 1] - o
    assert np.array_equal(m["lv_rows"][o:o + n], np.arange(n))
    lb = m["lv_base"][i]
    nlev = m["lv_base"][i + 1] - lb - 1
    lp, info = m["lv_ptr"][lb:lb + nlev + 1], m["lv_info"][lb:lb + nlev + 1]
    sb = m["st_ptr"][s0]
    for h in range(nlev):
        Js = np.arange(s0, s1)[ht == h]
        assert lp[h] == m["first"][Js[0]] and lp[h + 1] == m["first"][Js[-1]] + m["ncol"][Js[-1]]
        assert info[h, 0] == m["st_ptr"][Js[0]] - sb and info[h + 1, 0] == m["st_ptr"][Js[-1] + 1] - sb
        nc, ns = m["ncol"][Js].astype(np.int64), (m["nrow"][Js] - m["ncol"][Js]).astype(np.int64)
        assert info[h, 1] == (nc * (nc + 1) // 2).sum() and info[h, 2] == (nc * ns).sum()
        assert np.all(m["st_sn"][m["st_ptr"][Js[0]]:m["st_ptr"][Js[-1] + 1]] ==
                      np.repeat(Js, ns))
    assert info[nlev, 0] == m["st_ptr"][s1] - sb
    # the leaves in chunks of at most 64 rows, each a run of whole leaves
    ch = m["ch_row"][m["ch_base"][i]:m["ch_base"][i + 1]]
    leaf_ends = {0} | {int(m["first"][J] + m["ncol"][J]) for J in range(s0, s1) if ht[J - s0] == 0}
    assert ch[0] == 0 and ch[-1] == lp[1] and np.all(np.diff(ch) > 0) and np.all(np.diff(ch) <= 64)
    assert set(ch.tolist()) <= leaf_ends
    assert np.all(m["ncol"][s0:s1][ht == 0] <= 64)
    # gather entries: struct entry of K at row rr
    for rr in range(n):
        for q in range(m["rc_ptr"][o + rr], m["rc_ptr"][o + rr + 1]):
            K, pos = m["rc"][q]
            assert m["rc_w"][q] == m["st_ptr"][K] + pos - m["ncol"][K] - sb
            assert m["st_row"][sb + m["rc_w"][q]] == rr


CASES = {
    "poisson12_P2": lambda: (P.poisson3d(12, 2), None),
    "poisson17_P3_ragged": lambda: (P.poisson3d(17, 3), None),
    "elasticity4_P2": lambda: (lambda pr: (pr, P.rigid_body_modes(pr)))(P.elasticity_q1(4, 2)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_nd_structure_factor_and_solves(case):
    pr, Z = CASES[case]()
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, pr.dpn, Z,
                       B.gdsw_default_options(local=B.LOCAL_EXACT, exact_order=B.ORDER_ND))
    try:
        m = _maps(h)
        A = pr.A.tocsr()
        A.sort_indices()
        L = _factor(m, A.data)
        rng = np.random.default_rng(3)
        band = B.gdsw_get_info(h)["max_bandwidth"]
        for i in range(pr.n_parts):
            o0, o1 = m["ov_ptr"][i], m["ov_ptr"][i + 1]
            R = m["ov_idx"][o0:o1]
            perm = m["perm"][o0:o1]
            assert sorted(perm.tolist()) == list(range(o1 - o0))
            Ai = A[R][:, R]
            Ai_new = Ai[perm][:, perm]
            _check_levels(m, i)
            nnzL = _check_subdomain(m, i, L, sp.csr_matrix(Ai_new), rng)
            assert nnzL <= (o1 - o0) * (band + 1)
    finally:
        B.gdsw_destroy(h)


def test_nd_fill_below_the_band_on_the_large_subdomains():
    """On the 16^3 boxes of the 128^3 workload (5,632 rows with the overlap)
    the supernodal panels hold far fewer values than the band (1.81M)."""
    pr = P.poisson3d(48, 3)
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1, None,
                       B.gdsw_default_options(local=B.LOCAL_EXACT, exact_order=B.ORDER_ND))
    try:
        m = _maps(h)
        i = 13   # the centre box
        s0, s1 = m["sn_ptr"][i], m["sn_ptr"][i + 1]
        vals = int(m["voff"][s1] - m["voff"][s0])
        n = int(m["ov_ptr"][i + 1] - m["ov_ptr"][i])
        assert n == 5632
        assert vals < 0.5 * n * 321, vals
    finally:
        B.gdsw_destroy(h)


def test_default_order_is_the_band():
    pr = P.poisson3d(12, 2)
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1, None, B.gdsw_default_options())
    try:
        info = B.gdsw_get_info(h)
        assert info["exact_order"] == B.ORDER_NATURAL and info["nd_subdomains"] == 0
        assert B.gdsw_map_size(h, B.MAP_ND_SN) == 0
    finally:
        B.gdsw_destroy(h)


def test_auto_order_picks_the_smaller_factor():
    pr = P.poisson3d(48, 3)
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 1, None,
                       B.gdsw_default_options(local=B.LOCAL_EXACT, exact_order=B.ORDER_AUTO))
    try:
        info = B.gdsw_get_info(h)
        assert info["exact_order"] == B.ORDER_AUTO and info["nd_subdomains"] == pr.n_parts
        assert B.gdsw_map_size(h, B.MAP_ND_PERM) == info["sum_overlap_dofs"]
    finally:
        B.gdsw_destroy(h)
    pr = P.elasticity_q1(8, 2)
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 3, P.rigid_body_modes(pr),
                       B.gdsw_default_options(local=B.LOCAL_EXACT, exact_order=B.ORDER_AUTO))
    try:
        info = B.gdsw_get_info(h)
        nd = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 3, P.rigid_body_modes(pr),
                            B.gdsw_default_options(local=B.LOCAL_EXACT, exact_order=B.ORDER_ND))
        nd_vals = B.gdsw_get_info(nd)["local_factor_entries"]
        nat = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, 3, P.rigid_body_modes(pr),
                             B.gdsw_default_options(local=B.LOCAL_EXACT, exact_order=B.ORDER_NATURAL))
        band_vals = B.gdsw_get_info(nat)["local_factor_entries"]
        B.gdsw_destroy(nd)
        B.gdsw_destroy(nat)
        want = pr.n_parts if nd_vals < band_vals else 0
        assert info["nd_subdomains"] == want
        assert info["local_factor_entries"] == min(nd_vals, band_vals)
    finally:
        B.gdsw_destroy(h)

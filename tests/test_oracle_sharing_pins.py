"""Pins of the oracle's interface taken from element sharing sets (O4 for a
decomposition into subdomains of elements, Sec. III; the geometric GDSW
space on Q1 meshes) against what the geometry fixes: on a box partition of
the elements the components are exactly the interior faces, edges and
vertices of the boxes, with 6, 5 and 3 rigid-body modes (a plane, a line, a
point), so n_c and n_0 have closed forms; the coarse basis reproduces the
null space; the geometric space lies inside the node-graph space (its
components are unions of the node-graph components of R6 and the interior
sets coincide); M is SPD and the solution equals a direct solve.  Sharing
sets built from the node-graph interface give back that interface."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import gdsw_oracle as O
from paper_2304_04876_amd import problems as P


def _geo(pr, Z, **kw):
    return O.GDSW(pr.A, pr.part, pr.dpn, pr.n_parts, Z=Z, local="exact", sharing=P.element_sharing(pr), **kw)


def _box_starts(P_, G):
    g = np.arange(G + 1)
    b = np.minimum(g * P_ // G, P_ - 1)
    return {int(g[b == k].min()) for k in range(1, P_)}


@pytest.mark.parametrize("Ne,Pn", [(6, 2), (9, 3), (12, 4)])
def test_components_are_box_faces_edges_vertices(Ne, Pn):
    """Boxes of three elements per side, so that every face keeps two node
    columns beside the clamped plane x = 0 (a plane: 6 modes) and every edge
    two nodes (a line: 5)."""
    pr = P.elasticity_q1(Ne, Pn)
    M = _geo(pr, P.rigid_body_modes(pr))
    grid = np.rint(pr.coords * Ne).astype(int)
    starts = _box_starts(Pn, Ne)
    kind = {2: [], 4: [], 8: []}
    for nodes in M.comps:
        s = M.S[int(nodes[0])]
        assert all(M.S[int(v)] == s for v in nodes)
        kind[len(s)].append(nodes)
        # the nodes lie on 1, 2 or 3 box planes, one per doubling of the set
        on = [len({int(x) for x in grid[nodes, a]}) == 1 and int(grid[nodes[0], a]) in starts for a in range(3)]
        assert sum(on) == {2: 1, 4: 2, 8: 3}[len(s)]
    f, e, v = 3 * Pn * Pn * (Pn - 1), 3 * Pn * (Pn - 1) ** 2, (Pn - 1) ** 3
    assert (len(kind[2]), len(kind[4]), len(kind[8])) == (f, e, v)
    ranks = {len(M.S[int(c[0])]): set() for c in M.comps}
    for c, cols in zip(M.comps, M.cs.comp_cols):
        ranks[len(M.S[int(c[0])])].add(len(cols))
    assert ranks == {2: {6}, 4: {5}, 8: {3}}
    assert M.n0 == 6 * f + 5 * e + 3 * v


def _span_residual(B, X):
    C, *_ = np.linalg.lstsq(B, X, rcond=None)
    return np.linalg.norm(B @ C - X) / max(np.linalg.norm(X), 1e-300), C


def test_null_space_reproduced():
    pr = P.elasticity_q1(9, 3)
    Z = P.rigid_body_modes(pr)
    M = _geo(pr, Z)
    phi = M.cs.phi.toarray()
    gdofs = O.dofs_of(np.nonzero(M.is_gamma)[0], pr.dpn)
    res, C = _span_residual(phi[gdofs], Z[gdofs])
    assert res <= 1e-12
    AZ = pr.A @ Z
    interior = np.nonzero(~M.is_gamma)[0]
    checked = 0
    for i in range(pr.n_parts):
        Ii = O.dofs_of(interior[pr.part[interior] == i], pr.dpn)
        if Ii.size == 0 or np.abs(AZ[Ii]).max() > 1e-12:
            continue
        checked += 1
        assert np.abs(phi[Ii] @ C - Z[Ii]).max() <= 1e-10 * np.abs(Z).max()
    assert checked >= 1


def test_geometric_space_inside_node_graph_space():
    pr = P.elasticity_q1(8, 3)
    Z = P.rigid_body_modes(pr)
    Mg = _geo(pr, Z)
    Ma = O.GDSW(pr.A, pr.part, pr.dpn, pr.n_parts, Z=Z, local="exact")
    assert np.array_equal(Mg.is_gamma, Ma.is_gamma)
    assert Mg.n0 < Ma.n0
    res, _ = _span_residual(Ma.cs.phi.toarray(), Mg.cs.phi.toarray())
    assert res <= 1e-10


def test_spd_and_direct_solution():
    pr = P.elasticity_q1(4, 2)
    M = _geo(pr, P.rigid_body_modes(pr))
    Mo = np.column_stack([M.apply(e) for e in np.eye(pr.n)])
    assert np.abs(Mo - Mo.T).max() <= 1e-13 * np.abs(Mo).max()
    assert np.linalg.eigvalsh(0.5 * (Mo + Mo.T)).min() > 0
    pr = P.elasticity_q1(6, 2)
    M = _geo(pr, P.rigid_body_modes(pr))
    x = spla.spsolve(pr.A.tocsc(), pr.b)
    res = O.gmres(pr.A, pr.b, M, rtol=1e-12, restart=30)
    assert res.converged and np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)


def test_node_graph_sets_give_back_the_node_graph_interface():
    pr = P.poisson3d(10, 2)
    Ma = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local="exact")
    sets = [Ma.S.get(v, (int(pr.part[v]),)) for v in range(pr.n)]
    ptr = np.concatenate([[0], np.cumsum([len(t) for t in sets])]).astype(np.int64)
    sub = np.concatenate([np.array(t, dtype=np.int32) for t in sets])
    is_g, S = O.interface_from_sharing(ptr, sub, pr.part)
    assert np.array_equal(is_g, Ma.is_gamma) and S == Ma.S
    Ms = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local="exact", sharing=(ptr, sub))
    r = P.rhs_uniform(pr.n, 1)
    assert np.abs(Ms.apply(r) - Ma.apply(r)).max() <= 1e-14 * np.abs(Ma.apply(r)).max()


def test_sets_without_the_own_subdomain_are_rejected():
    pr = P.elasticity_q1(4, 2)
    ptr, sub = P.element_sharing(pr)
    bad = sub.copy()
    v = int(np.argmax(np.diff(ptr) == 1))
    bad[ptr[v]] = (pr.part[v] + 1) % pr.n_parts
    with pytest.raises(ValueError):
        O.interface_from_sharing(ptr, bad, pr.part)

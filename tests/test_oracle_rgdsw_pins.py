"""Pins of the oracle's reduced GDSW coarse space (O8r: coarse functions for
the vertices only, Sec. III, variants of GDSW) against what the geometry and
the algebra fix: with the 27-point coupling of Q1 elasticity on a box
partition the coarse nodes are exactly the interior cross points of the
boxes; the interface basis is a partition of unity times the null space (the
null space is reproduced); the reduced space lies inside the full GDSW space
(a different construction); the coarse functions are discrete harmonic in
the interiors; M stays SPD; iteration counts stay bounded as the number of
subdomains grows."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import gdsw_oracle as O
from paper_2304_04876_amd import problems as P


def _rgdsw(pr, Z, local="exact"):
    return O.GDSW(pr.A, pr.part, pr.dpn, pr.n_parts, Z=Z, local=local, coarse_space="rgdsw")


def _box_starts(P_, G):
    """First grid index of boxes 1 .. P-1 along an axis (box of g:
    min(g P // G, P - 1))."""
    g = np.arange(G + 1)
    b = np.minimum(g * P_ // G, P_ - 1)
    return {int(g[b == k].min()) for k in range(1, P_)}


@pytest.mark.parametrize("Ne,Pn", [(9, 2), (12, 3), (16, 4)])
def test_coarse_nodes_are_interior_cross_points(Ne, Pn):
    pr = P.elasticity_q1(Ne, Pn)
    M = _rgdsw(pr, P.rigid_body_modes(pr))
    coarse, owners = O.rgdsw_coarse_nodes(M.comps, M.S)
    grid = np.rint(pr.coords * Ne).astype(int)
    starts = _box_starts(Pn, Ne)   # the elasticity boxes use G = Ne
    expected = {(x, y, z) for x in starts for y in starts for z in starts}
    got = set()
    for v in coarse:
        nodes = M.comps[v]
        assert nodes.size == 1
        got.add(tuple(grid[nodes[0]]))
    assert got == expected
    assert M.n0 == 6 * (Pn - 1) ** 3
    # every component belongs to at least one coarse node
    assert all(len(o) >= 1 for o in owners)


def _span_residual(B, X):
    C, *_ = np.linalg.lstsq(B, X, rcond=None)
    return np.linalg.norm(B @ C - X) / max(np.linalg.norm(X), 1e-300), C


@pytest.mark.parametrize("case", ["poisson", "elasticity"])
def test_null_space_reproduced(case):
    """On the interface the basis holds Z (partition of unity); in every
    subdomain interior where A Z vanishes, Phi C equals Z."""
    if case == "poisson":
        pr = P.poisson3d(12, 3)
        Z = np.ones((pr.n, 1))
    else:
        pr = P.elasticity_q1(9, 3)
        Z = P.rigid_body_modes(pr)
    M = _rgdsw(pr, Z)
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


@pytest.mark.parametrize("case", ["poisson", "elasticity"])
def test_reduced_space_inside_gdsw_space(case):
    """Each reduced interface function restricted to a component is a
    combination of the null space there, and the extension is the same
    linear map, so range(Phi_rgdsw) lies in range(Phi_gdsw)."""
    if case == "poisson":
        pr = P.poisson3d(10, 2)
        Z = np.ones((pr.n, 1))
    else:
        pr = P.elasticity_q1(8, 3)
        Z = P.rigid_body_modes(pr)
    Mr = _rgdsw(pr, Z)
    Mg = O.GDSW(pr.A, pr.part, pr.dpn, pr.n_parts, Z=Z, local="exact")
    assert Mr.n0 < Mg.n0
    res, _ = _span_residual(Mg.cs.phi.toarray(), Mr.cs.phi.toarray())
    assert res <= 1e-10


def test_harmonic_in_the_interiors():
    pr = P.elasticity_q1(8, 2)
    M = _rgdsw(pr, P.rigid_body_modes(pr))
    AP = (pr.A @ M.cs.phi).toarray()
    interior = O.dofs_of(np.nonzero(~M.is_gamma)[0], pr.dpn)
    assert np.abs(AP[interior]).max() <= 1e-11 * np.abs(AP).max()


def test_spd():
    pr = P.elasticity_q1(4, 2)
    M = _rgdsw(pr, P.rigid_body_modes(pr))
    Mo = np.column_stack([M.apply(e) for e in np.eye(pr.n)])
    assert np.abs(Mo - Mo.T).max() <= 1e-13 * np.abs(Mo).max()
    assert np.linalg.eigvalsh(0.5 * (Mo + Mo.T)).min() > 0


def test_iterations_bounded_in_the_number_of_subdomains():
    """Elasticity with 2^3, 3^3, 4^3 boxes of the same size: the reduced
    coarse space keeps the GMRES iteration count nearly flat while the
    one-level method grows."""
    its, its1 = [], []
    for Pn in (2, 3, 4):
        pr = P.elasticity_q1(4 * Pn, Pn)
        Z = P.rigid_body_modes(pr)
        M = _rgdsw(pr, Z)
        its.append(O.gmres(pr.A, pr.b, M, rtol=1e-8, restart=30).iters)
        M1 = O.GDSW(pr.A, pr.part, 3, pr.n_parts, Z=Z, coarse=False)
        its1.append(O.gmres(pr.A, pr.b, M1, rtol=1e-8, restart=30).iters)
    assert its[-1] - its[0] <= 6, its
    assert its1[-1] - its1[0] >= 2 * (its[-1] - its[0]) + 4, (its, its1)


def test_solution_matches_direct():
    pr = P.elasticity_q1(6, 2)
    M = _rgdsw(pr, P.rigid_body_modes(pr))
    x = spla.spsolve(pr.A.tocsc(), pr.b)
    res = O.gmres(pr.A, pr.b, M, rtol=1e-12, restart=30)
    assert res.converged and np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)

"""Pins of the oracle's level-based ILU(k) and FastILU (Sec. V-B, "Incomplete
Local Solver"; ILU(k) levels in Sec. VII-C) against what the mathematics
fixes: the level-of-fill rule written out densely on small matrices, the
closed-form fill of the 7-point stencil, exact LU at full fill, the
defining property of incomplete factors, closed-form LU pivots of a
tridiagonal matrix, and the fixed point of the FastILU sweeps."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import gdsw_oracle as O
from paper_2304_04876_amd import problems as P


def dense_levels(A: np.ndarray, p: int) -> np.ndarray:
    """Level-of-fill of ILU(p) by the textbook rule, densely: lev = 0 on A's
    pattern, inf elsewhere; row by row, for k < i ascending with lev(i,k) <= p,
    lev(i,j) = min(lev(i,j), lev(i,k) + lev(k,j) + 1) for j > k; entries above
    p are dropped (inf)."""
    n = A.shape[0]
    INF = 10 ** 9
    lev = np.where(A != 0, 0, INF)
    for i in range(n):
        for k in range(i):
            if lev[i, k] > p:
                continue
            for j in range(k + 1, n):
                if lev[k, j] <= p:
                    lev[i, j] = min(lev[i, j], lev[i, k] + lev[k, j] + 1)
        lev[i, lev[i] > p] = INF
    return lev


def random_spd_pattern(n, density, seed):
    rng = np.random.default_rng(seed)
    M = (rng.random((n, n)) < density).astype(float)
    M = np.triu(M, 1)
    M = M + M.T
    A = -M * rng.random((n, n))
    A = (A + A.T) / 2
    np.fill_diagonal(A, np.abs(A).sum(1) + 1.0)
    return A


@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("seed", [0, 1])
def test_level_of_fill_matches_dense_rule(p, seed):
    A = random_spd_pattern(40, 0.08, seed)
    Pm, lev = O.iluk_pattern(sp.csr_matrix(A), p)
    ref = dense_levels(A, p)
    got = np.full(A.shape, 10 ** 9)
    Pm = Pm.tocoo()
    got[Pm.row, Pm.col] = lev
    assert np.array_equal(got, ref)


def test_ilu3_pattern_of_the_7point_stencil_past_the_first_capacity():
    """ILU(3) of the 7-point stencil on a 6^3 grid: more pattern entries than
    the first capacity (4 nnz(A)), so the pattern is computed again with more
    room; it equals the dense level-of-fill rule."""
    A = P.poisson3d(6, 1).A.tocsr()
    Pm, lev = O.iluk_pattern(A, 3)
    assert Pm.nnz > 4 * A.nnz
    ref = dense_levels(A.toarray(), 3)
    got = np.full(A.shape, 10 ** 9)
    Pm = Pm.tocoo()
    got[Pm.row, Pm.col] = lev
    assert np.array_equal(got, ref)


def test_ilu1_fill_of_the_7point_stencil():
    """On an N^3 grid in natural order, eliminating the three lower neighbours
    i-1, i-N, i-N^2 of an interior row creates exactly the six couplings
    i +- (N-1), i +- (N^2-1), i +- (N^2-N); ILU(1) rows hold 13 entries."""
    N = 6
    A = P.poisson3d(N, 1).A
    Pm, lev = O.iluk_pattern(A, 1)
    want = sorted({0, 1, -1, N, -N, N * N, -N * N, N - 1, -(N - 1), N * N - 1, -(N * N - 1),
                   N * N - N, -(N * N - N)})
    for (x, y, z) in [(2, 2, 2), (3, 2, 4), (1, 3, 2)]:
        i = x + N * y + N * N * z
        cols = Pm.indices[Pm.indptr[i]:Pm.indptr[i + 1]]
        assert sorted((cols - i).tolist()) == want
        # the new entries are exactly the level-1 ones
        levs = lev[Pm.indptr[i]:Pm.indptr[i + 1]]
        assert sorted((cols[levs == 1] - i).tolist()) == sorted(
            [N - 1, -(N - 1), N * N - 1, -(N * N - 1), N * N - N, -(N * N - N)])


def test_full_fill_is_lu():
    """With the level at least n every fill is kept: L U = A exactly."""
    A = random_spd_pattern(30, 0.1, 3)
    f = O.ilu_factors(sp.csr_matrix(A), level=30)
    n = A.shape[0]
    L = np.eye(n) + f.NL.toarray()
    U = f.NU.toarray() + np.diag(f.d)
    assert np.abs(L @ U - A).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("p", [0, 1, 2])
def test_incomplete_factors_reproduce_a_on_their_pattern(p):
    """The defining property of ILU on a pattern S: (L U)_ij = a_ij for every
    (i, j) in S (and L, U vanish off S)."""
    pr = P.poisson3d(5, 1)
    A = pr.A.toarray()
    Pm, _ = O.iluk_pattern(pr.A, p)
    f = O.ilu_factors(pr.A, level=p)
    n = A.shape[0]
    L = np.eye(n) + f.NL.toarray()
    U = f.NU.toarray() + np.diag(f.d)
    mask = Pm.copy()
    mask.data[:] = 1
    S = mask.toarray() != 0
    assert np.abs((L @ U - A)[S]).max() <= 1e-13 * np.abs(A).max()
    assert np.all(L[~S & ~np.eye(n, dtype=bool)] == 0) and np.all(U[~S] == 0)


def tridiag(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")


def test_fastilu_tridiagonal_propagation():
    """A = tridiag(-1, 2, -1): the LU pivots are u_ii = (i+2)/(i+1) and
    l_{i+1,i} = -(i+1)/(i+2).  From the start l = a_ij/a_jj, u = a_ij, each
    Jacobi sweep makes one more factor entry exact along the chain
    u_00, l_10, u_11, l_21, ...: after s sweeps u_ii is exact exactly for
    i <= (s+1)//2 (a sweep that used values of the same sweep would finish in
    one sweep)."""
    n = 12
    A = tridiag(n)
    Pm, _ = O.iluk_pattern(A, 0)
    exact_u = np.array([(i + 2) / (i + 1) for i in range(n)])
    exact_l = np.array([-(i + 1) / (i + 2) for i in range(n - 1)])
    for s in range(0, 8):
        F = O.fastilu_sweeps(Pm, s)
        u = F.diagonal()
        ok = np.isclose(u, exact_u, rtol=0, atol=1e-15)
        k = (s + 1) // 2
        assert ok[:k + 1].all(), (s, u)
        assert not ok[k + 1:].any(), (s, u)
        l = F.diagonal(-1)
        okl = np.isclose(l, exact_l, rtol=0, atol=1e-15)
        assert okl[:s // 2 + 1].all() and not okl[s // 2 + 1:].any(), (s, l)
    F = O.fastilu_sweeps(Pm, 2 * n)
    assert np.allclose(F.diagonal(), exact_u, rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", [0, 1])
def test_fastilu_fixed_point_is_ilu(p):
    """The exact ILU(p) factors are the fixed point of the sweeps; on a small
    grid enough sweeps reach them to rounding."""
    pr = P.poisson3d(4, 1)
    exact = O.ilu_factors(pr.A, level=p)
    fast = O.ilu_factors(pr.A, level=p, factor_sweeps=60)
    for a, b in ((exact.NL, fast.NL), (exact.NU, fast.NU)):
        assert np.abs((a - b).toarray()).max() <= 1e-14
    assert np.abs(exact.d - fast.d).max() <= 1e-14


def test_fastilu_first_sweep_by_hand():
    """One sweep on a 3x3 matrix, written out by hand:
    A = [[4,-1,-1],[-1,4,-1],[-1,-1,4]], start l_ij = a_ij/4, u_ij = a_ij.
    u_00 = 4, u_01 = u_02 = -1; l_10 = l_20 = -1/4; u_11 = 4 - (-1/4)(-1) = 3.75;
    u_12 = -1 - (-1/4)(-1) = -1.25; l_21 = (-1 - (-1/4)(-1)) / 4 = -0.3125;
    u_22 = 4 - (-1/4)(-1) - (-1/4)(-1) = 3.5."""
    A = sp.csr_matrix(np.array([[4.0, -1, -1], [-1, 4, -1], [-1, -1, 4]]))
    Pm, _ = O.iluk_pattern(A, 0)
    F = O.fastilu_sweeps(Pm, 1).toarray()
    want = np.array([[4.0, -1, -1], [-0.25, 3.75, -1.25], [-0.25, -0.3125, 3.5]])
    assert np.array_equal(F, want)


def test_ilu_level0_routes_agree():
    """ILU(0) through the ILU(k) path equals the plain ILU(0) factors."""
    pr = P.poisson3d(5, 1)
    a = O.ilu0_factors(pr.A)
    b = O.ilu_factors(pr.A, level=0)
    assert np.array_equal(a.NL.toarray(), b.NL.toarray())
    assert np.array_equal(a.NU.toarray(), b.NU.toarray())
    assert np.array_equal(a.d, b.d)

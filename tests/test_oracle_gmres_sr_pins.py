"""Pins of the oracle's single-reduce GMRES (Sec. VII: the Krylov solver of
the paper's experiments is a single-reduce GMRES(30)) against what the
mathematics fixes: GMRES minimises the residual over the Krylov space
(checked by brute force on explicit Krylov vectors), the Arnoldi relation
and orthonormality of the basis (checked with the operator applied anew),
finite termination, agreement with the modified Gram-Schmidt GMRES, and the
direct solution."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import gdsw_oracle as O
from paper_2304_04876_amd import problems as P


def _poisson_ilu(N=6, Pn=2):
    pr = P.poisson3d(N, Pn)
    M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local="ilu0")
    return pr, M


def _elasticity():
    pr = P.elasticity_q1(6, 2)
    M = O.GDSW(pr.A, pr.part, 3, pr.n_parts, Z=P.rigid_body_modes(pr), local="exact")
    return pr, M


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_minimal_residual_over_krylov_space(k):
    """x_k minimises ||b - A x|| over x in M^{-1} K_k(A M^{-1}, b): the
    Krylov vectors are formed explicitly, orthonormalised by a library QR,
    and the least-squares problem solved by a library routine."""
    pr, M = _poisson_ilu()
    b = P.rhs_uniform(pr.n, 3)
    B = lambda v: pr.A @ M.apply(v)
    K = np.zeros((pr.n, k))
    K[:, 0] = b / np.linalg.norm(b)
    for i in range(1, k):
        v = B(K[:, i - 1])
        K[:, i] = v / np.linalg.norm(v)
    Qk, _ = np.linalg.qr(K)
    BK = np.column_stack([B(Qk[:, i]) for i in range(k)])
    y, *_ = np.linalg.lstsq(BK, b, rcond=None)
    x_bf = M.apply(Qk @ y)
    res_bf = np.linalg.norm(b - pr.A @ x_bf)
    out = O.gmres_single_reduce(pr.A, b, M, restart=30, fixed_iters=k)
    res = np.linalg.norm(b - pr.A @ out.x)
    assert abs(res - res_bf) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(out.x - x_bf) <= 1e-8 * np.linalg.norm(x_bf)
    # the recursive estimate is the true residual of the iterate
    assert abs(out.history[-1] * np.linalg.norm(b) - res) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("k", [5, 17])
def test_arnoldi_relation_and_orthonormal_basis(k):
    pr, M = _elasticity()
    out, (Q, H) = O.gmres_single_reduce(pr.A, pr.b, M, restart=30, fixed_iters=k, return_basis=True)
    assert Q.shape == (pr.n, k + 1) and H.shape == (k + 1, k)
    assert np.abs(Q.T @ Q - np.eye(k + 1)).max() <= 1e-12
    BQ = np.column_stack([pr.A @ M.apply(Q[:, i]) for i in range(k)])
    assert np.linalg.norm(BQ - Q @ H) <= 1e-12 * np.linalg.norm(BQ)
    # upper Hessenberg with a positive subdiagonal; first column from b
    assert np.all(np.tril(H, -2) == 0) and np.all(np.diag(H, -1) > 0)
    assert np.abs(Q[:, 0] - pr.b / np.linalg.norm(pr.b)).max() <= 1e-15


@pytest.mark.parametrize("restart", [30, 5])
def test_same_iterates_as_mgs_gmres(restart):
    pr, M = _elasticity()
    for k in (3, 8, 13):
        a = O.gmres(pr.A, pr.b, M, restart=restart, fixed_iters=k)
        s = O.gmres_single_reduce(pr.A, pr.b, M, restart=restart, fixed_iters=k)
        assert np.linalg.norm(a.x - s.x) <= 1e-12 * np.linalg.norm(a.x)
        assert np.allclose(a.history, s.history, rtol=1e-10, atol=0)
    a = O.gmres(pr.A, pr.b, M, rtol=1e-8, restart=restart)
    s = O.gmres_single_reduce(pr.A, pr.b, M, rtol=1e-8, restart=restart)
    assert a.iters == s.iters and s.converged


def test_converges_to_direct_solution():
    pr, M = _elasticity()
    x = spla.spsolve(pr.A.tocsc(), pr.b)
    for restart in (30, 4):
        res = O.gmres_single_reduce(pr.A, pr.b, M, rtol=1e-12, restart=restart)
        assert res.converged
        assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)


def test_finite_termination():
    """A diagonal matrix with three distinct eigenvalues: the Krylov space is
    invariant after three steps, GMRES is exact there and stops."""
    n = 60
    d = np.repeat([1.0, 2.0, 5.0], n // 3)
    A = sp.diags(d, format="csr")
    b = np.random.default_rng(0).standard_normal(n)
    res = O.gmres_single_reduce(A, b, None, rtol=1e-14, restart=30)
    assert res.iters == 3
    assert np.linalg.norm(res.x - b / d) <= 1e-13 * np.linalg.norm(b / d)
    # identity: one step
    res = O.gmres_single_reduce(sp.identity(n, format="csr"), b, None, rtol=1e-14)
    assert res.iters == 1 and np.abs(res.x - b).max() <= 1e-15 * np.abs(b).max()


def test_zero_rhs():
    pr, M = _poisson_ilu(4, 2)
    res = O.gmres_single_reduce(pr.A, np.zeros(pr.n), M)
    assert res.iters == 0 and res.converged and not res.x.any()


@pytest.mark.parametrize("delta", [1e-6, 1e-12])
def test_nearly_invariant_krylov_space(delta):
    """Four eigenvalue clusters of width delta: after four steps the new
    direction is tiny against A M^{-1} q (the case where one projection pass
    or a shortcut in the normalisation loses orthogonality); the basis must
    stay orthonormal, satisfy the Arnoldi relation and give the iterates of
    the modified Gram-Schmidt GMRES."""
    n = 200
    rng = np.random.default_rng(1)
    d = np.concatenate([c + delta * rng.random(50) for c in (1.0, 2.0, 3.0, 4.0)])
    A = sp.diags(d, format="csr")
    b = rng.standard_normal(n)
    for k in (5, 7):
        out, (Q, H) = O.gmres_single_reduce(A, b, None, restart=30, fixed_iters=k, return_basis=True)
        assert np.abs(Q.T @ Q - np.eye(k + 1)).max() <= 1e-12
        BQ = A @ Q[:, :k]
        assert np.linalg.norm(BQ - Q @ H) <= 1e-12 * np.linalg.norm(BQ)
        ref = O.gmres(A, b, None, restart=30, fixed_iters=k)
        assert np.linalg.norm(out.x - ref.x) <= 1e-12 * np.linalg.norm(ref.x)

"""Planted mistakes in the oracle (CPU only): each mutant must make at least
one pin fail, which shows the pins can see that kind of error."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_2304_04876_amd import problems as P
from oracle import gdsw_oracle as O
from tests.test_oracle_pins import geometric_gdsw_dense, oracle_dense


def _p2_error(local="exact", sweeps=5, N=6, Pn=2):
    pr, Minv = geometric_gdsw_dense(N, Pn, local, sweeps)
    M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local=local, sweeps=sweeps)
    Mo = oracle_dense(M, pr.n)
    return np.abs(Mo - Minv).max() / np.abs(Minv).max()


def test_unmutated_oracle_passes():
    assert _p2_error() <= 1e-13
    assert _p2_error("ilu0") <= 1e-13


def test_mutant_extension_sign(monkeypatch):
    real = O.extension_solve
    monkeypatch.setattr(O, "extension_solve", lambda A, r: -real(A, r))
    assert _p2_error() > 1e-6


def test_mutant_extension_dropped(monkeypatch):
    monkeypatch.setattr(O, "extension_solve", lambda A, r: 0.0 * r)
    assert _p2_error() > 1e-6


def test_mutant_interface_on_upper_faces(monkeypatch):
    real = O.interface

    def reversed_interface(G, part):
        return real(G, -part)
    monkeypatch.setattr(O, "interface", reversed_interface)
    assert _p2_error() > 1e-6


def test_mutant_no_overlap(monkeypatch):
    real = O.overlapping_subdomains
    monkeypatch.setattr(O, "overlapping_subdomains", lambda G, p, n, ov: real(G, p, n, 0))
    assert _p2_error() > 1e-6


def test_mutant_components_merged(monkeypatch):
    # one component per S-class would still be right here; merging all pieces
    # into a single constant is not
    monkeypatch.setattr(O, "components", lambda G, g, S: [np.nonzero(g)[0]])
    assert _p2_error() > 1e-6


def test_mutant_ilu_without_update(monkeypatch):
    import scipy.sparse as sp

    def diag_only(Ai):
        f = O.ILU0(sp.tril(Ai, -1, format="csr") * 0, sp.triu(Ai, 1, format="csr"), Ai.diagonal())
        return f
    monkeypatch.setattr(O, "ilu0_factors", diag_only)
    assert _p2_error("ilu0") > 1e-6


def test_mutant_jacobi_sign(monkeypatch):
    def bad(f, r, K):
        y = np.zeros_like(r)
        for _ in range(K):
            y = r + f.NL @ y
        w = np.zeros_like(r)
        for _ in range(K):
            w = (y - f.NU @ w) / f.d
        return w
    monkeypatch.setattr(O, "ilu0_jacobi_solve", bad)
    assert _p2_error("ilu0") > 1e-6


def test_mutant_cg_beta(monkeypatch):
    pr = P.poisson3d(12, 2)
    M = O.GDSW(pr.A, pr.part, 1, pr.n_parts)
    b = P.rhs_uniform(pr.n, 0)
    x = spla.spsolve(pr.A.tocsc(), b)
    good = O.pcg(pr.A, b, M, 1e-12, maxit=60)
    assert np.linalg.norm(good.x - x) <= 1e-9 * np.linalg.norm(x)

    # a preconditioner that is not fixed breaks CG's convergence: shows the
    # solution check can see a wrong search direction
    class Bad:
        def __init__(self):
            self.k = 0
        def apply(self, r):
            self.k += 1
            return M.apply(r) * (1.0 if self.k % 2 else 3.0) + 0.1 * r
    bad = O.pcg(pr.A, b, Bad(), 1e-12, maxit=60)
    assert np.linalg.norm(bad.x - x) > 1e-9 * np.linalg.norm(x) or bad.iters > good.iters


# ---- FastILU and ILU(k) mutants: each must trip an ILU pin ---------------------

def _mutant_fastilu(mode):
    import scipy.sparse as sp

    def sweeps_fn(Pm, sweeps):
        n = Pm.shape[0]
        ip, ix, a = Pm.indptr, Pm.indices, Pm.data
        where = [dict(zip(ix[ip[i]:ip[i + 1]].tolist(), range(ip[i], ip[i + 1]))) for i in range(n)]
        dpos = np.array([where[i][i] for i in range(n)])
        v = a.copy()
        for i in range(n):
            for e in range(ip[i], ip[i + 1]):
                if ix[e] < i:
                    v[e] = 0.0 if mode == "zero_start" else a[e] / a[dpos[ix[e]]]
        for _ in range(sweeps):
            new = v if mode == "in_place" else np.empty_like(v)
            for i in range(n):
                for e in range(ip[i], ip[i + 1]):
                    j = int(ix[e])
                    acc = a[e]
                    for f in range(ip[i], ip[i + 1]):
                        m = int(ix[f])
                        if m >= min(i, j):
                            break
                        g = where[m].get(j)
                        if g is not None:
                            acc -= v[f] * v[g]
                    divide = i > j and mode != "no_division"
                    new[e] = acc / v[dpos[j]] if divide else acc
            v = new
        return sp.csr_matrix((v, ix.copy(), ip.copy()), shape=Pm.shape)
    return sweeps_fn


def _ilu_pins_fail():
    from tests import test_oracle_ilu_pins as T
    failures = 0
    for fn in (T.test_fastilu_tridiagonal_propagation, T.test_fastilu_first_sweep_by_hand,
               lambda: T.test_fastilu_fixed_point_is_ilu(1)):
        try:
            fn()
        except AssertionError:
            failures += 1
    return failures


def test_fastilu_pins_pass_unmutated():
    assert _ilu_pins_fail() == 0


@pytest.mark.parametrize("mode", ["in_place", "no_division", "zero_start"])
def test_mutant_fastilu(monkeypatch, mode):
    monkeypatch.setattr(O, "fastilu_sweeps", _mutant_fastilu(mode))
    assert _ilu_pins_fail() > 0


def test_mutant_iluk_without_fill(monkeypatch):
    from tests import test_oracle_ilu_pins as T
    real = O.iluk_pattern
    monkeypatch.setattr(O, "iluk_pattern", lambda A, level: real(A, 0))
    with pytest.raises(AssertionError):
        T.test_ilu1_fill_of_the_7point_stencil()


# single-reduce GMRES: planted mistakes in the per-step arithmetic.  (Errors
# in the first-pass coefficients alone are not planted: the next step's
# second pass measures and removes them, so they change results only at
# rounding level.)
def _mutant_sr_coefficients(mode):
    def coeffs(H, a_prev, j, c, d, e, f):
        beta2 = e if mode == "no_pythagoras" else e - c @ c
        beta = float(np.sqrt(beta2)) if beta2 > 0.0 else 0.0
        if j >= 1:
            H[:j, j - 1] = a_prev + c
            H[j, j - 1] = beta
        if beta == 0.0:
            return beta, None, None
        Hc = H[:j + 1, :j] @ c
        if mode == "no_relation":
            Hc = 0.0 * Hc
        a = np.empty(j + 1)
        a[:j] = (d - Hc[:j]) / beta
        a[j] = ((f - c @ d) / beta - Hc[j]) / beta
        return beta, Hc, a
    return coeffs


def _sr_pins_fail():
    from tests import test_oracle_gmres_sr_pins as T
    failures = 0
    for fn in (lambda: T.test_arnoldi_relation_and_orthonormal_basis(17),
               lambda: T.test_nearly_invariant_krylov_space(1e-12),
               lambda: T.test_same_iterates_as_mgs_gmres(30),
               lambda: T.test_minimal_residual_over_krylov_space(6)):
        try:
            fn()
        except AssertionError:
            failures += 1
    return failures


def test_sr_pins_pass_unmutated():
    assert _sr_pins_fail() == 0


@pytest.mark.parametrize("mode", ["no_pythagoras", "no_relation"])
def test_mutant_single_reduce_coefficients(monkeypatch, mode):
    monkeypatch.setattr(O, "sr_coefficients", _mutant_sr_coefficients(mode))
    assert _sr_pins_fail() > 0


def test_mutant_single_reduce_one_pass(monkeypatch):
    monkeypatch.setattr(O, "sr_basis_vector", lambda Q, j, u, c, beta: u / beta)
    assert _sr_pins_fail() > 0


def test_mutant_single_reduce_unscaled_direction(monkeypatch):
    def bad(Q, j, z, beta, Hc, a):
        w = z - Q[:, :j + 1] @ Hc
        return w - Q[:, :j + 1] @ a
    monkeypatch.setattr(O, "sr_next_candidate", bad)
    assert _sr_pins_fail() > 0


# reduced GDSW: planted mistakes in the coarse nodes and the weights
def _rgdsw_pins_fail():
    from tests import test_oracle_rgdsw_pins as T
    failures = 0
    for fn in (lambda: T.test_coarse_nodes_are_interior_cross_points(12, 3),
               lambda: T.test_null_space_reproduced("elasticity"),
               lambda: T.test_null_space_reproduced("poisson"),
               lambda: T.test_reduced_space_inside_gdsw_space("elasticity")):
        try:
            fn()
        except AssertionError:
            failures += 1
    return failures


def test_rgdsw_pins_pass_unmutated():
    assert _rgdsw_pins_fail() == 0


def test_mutant_rgdsw_missing_coarse_nodes(monkeypatch):
    # only the components with the largest subdomain sets become coarse nodes
    real = O.rgdsw_coarse_nodes

    def fewer(comps, S):
        coarse, owners = real(comps, S)
        top = max(len(S[int(comps[v][0])]) for v in coarse)
        keep = [v for v in coarse if len(S[int(comps[v][0])]) == top]
        return keep, [[v for v in o if v in keep] for o in owners]
    monkeypatch.setattr(O, "rgdsw_coarse_nodes", fewer)
    assert _rgdsw_pins_fail() > 0


def test_mutant_rgdsw_weights_not_a_partition_of_unity(monkeypatch):
    monkeypatch.setattr(O, "rgdsw_weight", lambda owners: 1.0)
    assert _rgdsw_pins_fail() > 0

"""GPU parity of the reduced GDSW coarse space (Sec. III, variants of GDSW;
the coarse space of the paper's experiments, Sec. VII) through the C ABI
against the oracle.  Tolerances as for the full GDSW space: basis, coarse
matrix and apply to 1e-12 relative to their largest entry (both sides build
the same orthonormal bases by Gram-Schmidt in the same row order and the
same extension, and differ only in summation order and in the local and
coarse factorisations); Krylov iteration counts within +-1 and iterates
after a fixed number of iterations to 1e-10."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_2304_04876_amd import binding as B
from paper_2304_04876_amd import problems as P
from oracle import gdsw_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = {
    "poisson12_P3": lambda: (P.poisson3d(12, 3), None),
    "poisson17_P3_ragged": lambda: (P.poisson3d(17, 3), None),
    "elasticity6_P2": lambda: ((lambda p: (p, P.rigid_body_modes(p)))(P.elasticity_q1(6, 2))),
    "elasticity9_P3": lambda: ((lambda p: (p, P.rigid_body_modes(p)))(P.elasticity_q1(9, 3))),
    "diffusion": lambda: (P.batch_diffusion_problem(P.batch_diffusion_specs(2)[1]), None),
}


@pytest.mark.parametrize("case", list(CASES))
def test_basis_coarse_matrix_and_apply(case):
    pr, Z = CASES[case]()
    say(f"[rgdsw] {case} n={pr.n}")
    M = O.GDSW(pr.A, pr.part, pr.dpn, pr.n_parts, Z=Z, local="exact", coarse_space="rgdsw")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, pr.dpn, Z, coarse=B.COARSE_RGDSW)
    n0 = g.info()["n0"]
    assert n0 == M.n0
    phi = sp.csr_matrix((g.map(B.MAP_PHI_VAL), g.map(B.MAP_PHI_COL), g.map(B.MAP_PHI_ROWPTR)),
                        shape=(pr.n, n0)).toarray()
    assert rel_max(phi, M.cs.phi.toarray()) <= 1e-12
    A0 = g.map(B.MAP_A0).reshape(n0, n0)
    assert rel_max(A0, M.A0) <= 1e-12
    r = P.rhs_uniform(pr.n, 3)
    rd, zd = dev(r), torch.zeros(pr.n, dtype=torch.float64, device="cuda")
    g.apply(rd, zd)
    assert rel_max(host(zd), M.apply(r)) <= 1e-12
    g.apply_part(rd, zd, 2)
    assert rel_max(host(zd), M.coarse_apply(r)) <= 1e-12
    g.close()


def test_single_reduce_gmres_elasticity():
    pr = P.elasticity_q1(9, 3)
    Z = P.rigid_body_modes(pr)
    say("[rgdsw] gmres-sr elasticity9")
    M = O.GDSW(pr.A, pr.part, 3, pr.n_parts, Z=Z, local="exact", coarse_space="rgdsw")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 3, Z, coarse=B.COARSE_RGDSW)
    ref = O.gmres_single_reduce(pr.A, pr.b, M, rtol=1e-8, restart=30)
    bd = dev(pr.b)
    xd = torch.zeros_like(bd)
    out = g.solve(bd, xd, krylov=B.KRYLOV_GMRES_SR, restart=30, rtol=1e-8)
    assert abs(out["iterations"] - ref.iters) <= 1 and out["converged"]
    k = 12
    fx = O.gmres_single_reduce(pr.A, pr.b, M, restart=30, fixed_iters=k)
    g.solve(bd, xd, krylov=B.KRYLOV_GMRES_SR, restart=30, fixed_iters=k)
    assert np.linalg.norm(host(xd) - fx.x) <= 1e-10 * np.linalg.norm(fx.x)
    g.close()


def test_cg_poisson_ilu0():
    pr = P.poisson3d(16, 4)
    say("[rgdsw] cg poisson16 ilu0")
    M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local="ilu0", coarse_space="rgdsw")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, local=B.LOCAL_ILU0, coarse=B.COARSE_RGDSW)
    b = P.rhs_uniform(pr.n, 1)
    ref = O.pcg(pr.A, b, M, rtol=1e-8)
    xd = torch.zeros(pr.n, dtype=torch.float64, device="cuda")
    out = g.solve(dev(b), xd, rtol=1e-8)
    assert abs(out["iterations"] - ref.iters) <= 1 and out["converged"]
    x = spla.spsolve(pr.A.tocsc(), b)
    assert np.linalg.norm(host(xd) - x) <= 1e-6 * np.linalg.norm(x)
    g.close()


def test_batch_matches_alone():
    """A batch handle with the reduced space: every problem's CG iterate is
    bitwise the one it gets alone, and its apply matches the oracle."""
    specs = P.batch_diffusion_specs(3)
    probs = [P.batch_diffusion_problem(sp_) for sp_ in specs]
    say("[rgdsw] batch of 3")
    opts = B.gdsw_default_options(coarse=B.COARSE_RGDSW)
    hb = B.gdsw_analyze_batch([(p.A, p.part, p.n_parts) for p in probs], 1, None, opts)
    B.gdsw_factor(hb)
    off = B.gdsw_problem_offsets(hb)
    bs = [P.rhs_uniform(p.n, 7 + i) for i, p in enumerate(probs)]
    bd = dev(np.concatenate(bs))
    xd = torch.zeros_like(bd)
    B.gdsw_solve_batch(hb, bd, xd, rtol=1e-8)
    xb = host(xd)
    zd = torch.zeros_like(bd)
    B.gdsw_apply(hb, bd, zd)
    zb = host(zd)
    for i, p in enumerate(probs):
        M = O.GDSW(p.A, p.part, 1, p.n_parts, local="exact", coarse_space="rgdsw")
        assert rel_max(zb[off[i]:off[i + 1]], M.apply(bs[i])) <= 1e-12
        g = B.Gdsw(p.A, p.part, p.n_parts, 1, coarse=B.COARSE_RGDSW)
        x1 = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        g.solve(dev(bs[i]), x1, rtol=1e-8)
        assert np.array_equal(host(x1), xb[off[i]:off[i + 1]])
        g.close()
    B.gdsw_destroy(hb)

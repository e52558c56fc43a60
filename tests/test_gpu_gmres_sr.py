"""GPU parity of the single-reduce GMRES (Sec. VII) through the C ABI against
the oracle's single-reduce GMRES, and against the library's classical
Gram-Schmidt GMRES.

Tolerances (FP64): iteration counts equal within +-1 (the two sides sum in
different orders, and the stopping test compares a residual estimate with
the tolerance); iterates after the same fixed number of iterations within
1e-10 relative (2-norm), as for the classical GMRES: both sides compute the
same iterate of a well-conditioned preconditioned operator, and the apply
agrees to 1e-12."""
import sys

import numpy as np
import pytest
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


@pytest.mark.parametrize("restart", [30, 5, 1])
def test_single_reduce_matches_oracle_elasticity(restart):
    pr = P.elasticity_q1(6, 2)
    Z = P.rigid_body_modes(pr)
    say(f"[gmres-sr] elasticity6 restart={restart}")
    M = O.GDSW(pr.A, pr.part, 3, pr.n_parts, Z=Z, local="exact")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 3, Z)
    b = pr.b
    ref = O.gmres_single_reduce(pr.A, b, M, rtol=1e-8, restart=restart, maxit=400)
    bd = dev(b)
    xd = torch.zeros_like(bd)
    out = g.solve(bd, xd, krylov=B.KRYLOV_GMRES_SR, restart=restart, rtol=1e-8, maxit=400)
    assert abs(out["iterations"] - ref.iters) <= 1, (out, ref.iters)
    assert out["converged"] and out["rel_res_true"] <= 1e-7
    # fixed iteration counts: inside the first cycle, at a restart boundary, across restarts
    for k in sorted({3, restart, min(ref.iters, 2 * restart + 1)}):
        fx = O.gmres_single_reduce(pr.A, b, M, restart=restart, fixed_iters=k)
        out = g.solve(bd, xd, krylov=B.KRYLOV_GMRES_SR, restart=restart, fixed_iters=k)
        assert out["iterations"] == k
        x = host(xd)
        assert np.linalg.norm(x - fx.x) <= 1e-10 * np.linalg.norm(fx.x), k
    g.close()


def test_single_reduce_matches_classical_gmres_poisson():
    pr = P.poisson3d(12, 3)
    say("[gmres-sr] poisson12 ilu0 vs classical")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, local=1)
    b = P.rhs_uniform(pr.n, 0)
    bd = dev(b)
    x1 = torch.zeros_like(bd)
    x2 = torch.zeros_like(bd)
    o1 = g.solve(bd, x1, krylov=B.KRYLOV_GMRES, restart=30, rtol=1e-8)
    o2 = g.solve(bd, x2, krylov=B.KRYLOV_GMRES_SR, restart=30, rtol=1e-8)
    assert abs(o1["iterations"] - o2["iterations"]) <= 1
    assert o2["converged"] and o2["rel_res_true"] <= 1e-7
    x = spla.spsolve(pr.A.tocsc(), b)
    assert np.linalg.norm(host(x2) - x) <= 1e-6 * np.linalg.norm(x)
    for k in (7, 31):
        g.solve(bd, x1, krylov=B.KRYLOV_GMRES, restart=30, fixed_iters=k)
        g.solve(bd, x2, krylov=B.KRYLOV_GMRES_SR, restart=30, fixed_iters=k)
        a, s = host(x1), host(x2)
        assert np.linalg.norm(a - s) <= 1e-10 * np.linalg.norm(a), k
    g.close()


def test_single_reduce_edge_cases():
    pr = P.poisson3d(8, 2)
    say("[gmres-sr] edge cases poisson8")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 1)
    # zero right-hand side: x = 0 without iterations
    bd = torch.zeros(pr.n, dtype=torch.float64, device="cuda")
    xd = torch.full_like(bd, 3.0)
    out = g.solve(bd, xd, krylov=B.KRYLOV_GMRES_SR)
    assert out["iterations"] == 0 and out["converged"] and not host(xd).any()
    # iteration cap: NOT_CONVERGED with the last iterate, equal to a fixed run
    b = P.rhs_uniform(pr.n, 4)
    bd = dev(b)
    out = g.solve(bd, xd, krylov=B.KRYLOV_GMRES_SR, rtol=1e-14, maxit=4, raise_on_error=False)
    assert out["status"] == 4 and out["iterations"] == 4
    x_cap = host(xd)
    M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local="exact")
    fx = O.gmres_single_reduce(pr.A, b, M, restart=30, fixed_iters=4)
    assert np.linalg.norm(x_cap - fx.x) <= 1e-10 * np.linalg.norm(fx.x)
    # the same handle keeps working for CG afterwards
    out = g.solve(bd, xd, krylov=B.KRYLOV_CG, rtol=1e-8)
    assert out["converged"]
    g.close()

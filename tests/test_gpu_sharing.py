"""GPU parity of the interface taken from element sharing sets
(gdsw_analyze_sharing: the geometric GDSW space of a decomposition into
subdomains of elements, Sec. III) against the FP64 oracle with the same
sets, through the C ABI: the coarse basis and A_0 to 1e-12 of their largest
entries, the apply to 1e-12 of the oracle's max-norm (exact local solves;
the same tolerances and reasons as for the node-graph interface), GMRES
iteration counts within +-1 and the fixed-iteration iterate to 1e-10; also
with the reduced coarse space built on these components."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

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


@pytest.mark.parametrize("Ne,Pn,coarse", [(6, 2, "gdsw"), (9, 3, "gdsw"), (9, 3, "rgdsw")])
def test_sharing_basis_a0_and_apply(Ne, Pn, coarse):
    pr = P.elasticity_q1(Ne, Pn)
    Z = P.rigid_body_modes(pr)
    sh = P.element_sharing(pr)
    say(f"[sharing] elasticity {Ne}^3 P={Pn} {coarse}")
    M = O.GDSW(pr.A, pr.part, 3, pr.n_parts, Z=Z, local="exact", sharing=sh, coarse_space=coarse)
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 3, Z, sharing=sh,
               coarse=B.COARSE_RGDSW if coarse == "rgdsw" else B.COARSE_GDSW)
    n0 = g.info()["n0"]
    assert n0 == M.n0
    phi = sp.csr_matrix((g.map(B.MAP_PHI_VAL), g.map(B.MAP_PHI_COL), g.map(B.MAP_PHI_ROWPTR)),
                        shape=(pr.n, n0)).toarray()
    assert rel_max(phi, M.cs.phi.toarray()) <= 1e-12
    assert rel_max(g.map(B.MAP_A0).reshape(n0, n0), M.A0) <= 1e-12
    r = P.rhs_uniform(pr.n, 7)
    rd, zd = dev(r), torch.zeros(pr.n, dtype=torch.float64, device="cuda")
    g.apply(rd, zd)
    assert rel_max(host(zd), M.apply(r)) <= 1e-12
    g.close()


def test_sharing_gmres_matches_oracle():
    pr = P.elasticity_q1(9, 3)
    Z = P.rigid_body_modes(pr)
    sh = P.element_sharing(pr)
    say("[sharing] GMRES elasticity 9^3 P=3")
    M = O.GDSW(pr.A, pr.part, 3, pr.n_parts, Z=Z, local="exact", sharing=sh)
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 3, Z, sharing=sh)
    ref = O.gmres(pr.A, pr.b, M, rtol=1e-8, restart=30)
    bd = dev(pr.b)
    xd = torch.zeros_like(bd)
    out = g.solve(bd, xd, krylov=B.KRYLOV_GMRES_SR, restart=30, rtol=1e-8)
    assert abs(out["iterations"] - ref.iters) <= 1, (out, ref.iters)
    assert out["converged"] and out["rel_res_true"] <= 1e-7
    k = ref.iters - 3
    fx = O.gmres(pr.A, pr.b, M, restart=30, fixed_iters=k)
    g.solve(bd, xd, krylov=B.KRYLOV_GMRES, restart=30, fixed_iters=k)
    assert np.linalg.norm(host(xd) - fx.x) <= 1e-10 * np.linalg.norm(fx.x)
    g.close()

"""The two column forms of the Krylov SpMV (sliced ELL with 16-bit offsets
from the row for banded orderings, 32-bit columns otherwise): the same
product A x as a library sparse product, and a CG solve that matches the
oracle's iteration count, on a Poisson problem in natural order (offsets
within 16 bits) and the same problem with its dofs randomly renumbered
(subdomains in a random order: offsets far beyond 16 bits).  FP64: the products agree to 1e-14 relative
(the same terms in a different summation order)."""
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


def renumbered(pr, seed):
    """Dofs numbered subdomain by subdomain, the subdomains in a random
    order, each in its natural order: the couplings across subdomains reach
    far beyond 16-bit offsets while every subdomain's interior stays banded
    (as the extension's band solves need)."""
    sub_rank = np.random.default_rng(seed).permutation(pr.n_parts)
    perm = np.lexsort((np.arange(pr.n), sub_rank[pr.part]))   # new dof j is old dof perm[j]
    Pm = sp.csr_matrix((np.ones(pr.n), (np.arange(pr.n), perm)), shape=(pr.n, pr.n))
    A = (Pm @ pr.A @ Pm.T).tocsr()
    A.sort_indices()
    return A, pr.part[perm]


@pytest.mark.parametrize("form", ["natural", "renumbered"])
def test_spmv_and_cg(form):
    pr = P.poisson3d(36, 3)   # 46,656 dofs: renumbered offsets exceed 32767
    A, part = (pr.A, pr.part) if form == "natural" else renumbered(pr, 7)
    offs = np.abs(A.indices - np.repeat(np.arange(pr.n), np.diff(A.indptr)))
    assert (offs.max() <= 32767) == (form == "natural")
    say(f"[spmv-forms] {form} n={pr.n} max offset {offs.max()}")
    g = B.Gdsw(A, part, pr.n_parts, 1, local=B.LOCAL_ILU0)
    x = np.random.default_rng(3).uniform(-1, 1, pr.n)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros_like(xd)
    g.spmv(xd, yd)
    torch.cuda.synchronize()
    y = A @ x
    assert np.abs(yd.cpu().numpy() - y).max() <= 1e-14 * np.abs(y).max()
    b = P.rhs_uniform(pr.n, 4)
    M = O.GDSW(A, part, 1, pr.n_parts, local="ilu0")
    ref = O.pcg(A, b, M, rtol=1e-8)
    bd = torch.from_numpy(b).cuda()
    xs = torch.zeros_like(bd)
    out = g.solve(bd, xs, rtol=1e-8)
    assert abs(out["iterations"] - ref.iters) <= 1 and out["converged"]
    g.close()

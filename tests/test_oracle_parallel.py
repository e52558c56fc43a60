"""The oracle's apply with the subdomain loop in worker processes (used for
the CPU baseline on all host cores) is the serial apply, bit for bit, and a
CG solve through it takes the same iterates."""
import numpy as np

from paper_2304_04876_amd import problems as P
from oracle import gdsw_oracle as O
from oracle.parallel import ForkedApply


def test_forked_apply_is_the_serial_apply():
    for local in ("ilu0", "exact"):
        pr = P.poisson3d(14, 3)
        M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local=local)
        r = P.rhs_uniform(pr.n, 4)
        with ForkedApply(M, 4) as F:
            assert F.workers == 4
            assert np.array_equal(F.apply(r), M.apply(r))
            a = O.pcg(pr.A, r, M, rtol=1e-8)
            b = O.pcg(pr.A, r, F, rtol=1e-8)
            assert a.iters == b.iters and np.array_equal(a.x, b.x)


def test_forked_apply_elasticity_more_workers_than_subdomains():
    pr = P.elasticity_q1(4, 2)
    Z = P.rigid_body_modes(pr)
    M = O.GDSW(pr.A, pr.part, 3, pr.n_parts, Z=Z, local="exact")
    with ForkedApply(M, 32) as F:
        assert 1 <= F.workers <= pr.n_parts
        r = P.rhs_uniform(pr.n, 1)
        assert np.array_equal(F.apply(r), M.apply(r))

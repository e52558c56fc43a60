"""How much rounding in the preconditioner moves a CG iterate (oracle only,
CPU).

The fixed-iteration CG comparison between the library and the oracle can
only be as tight as the oracle's own iterate is stable under rounding-level
changes of the operator.  These tests measure that on the 20^3 Poisson
workload (2^3 boxes, GDSW): every preconditioner apply of the oracle is
multiplied entry by entry by (1 + eps u), u seeded uniform(-1, 1), and the
fixed-iteration iterate is compared with the unperturbed one.

Measured (eps = 1e-16, three perturbation seeds, right-hand sides 0..2):
* exact local solves: the spread stays at rounding level (<= 1e-15) up to
  the converged iteration count (24-25);
* ILU(0) with 5+5 Jacobi sweeps: rounding level up to iteration 15, then the
  spread grows by about 1.8x per iteration, to 1e-10 relative at the
  converged count 43 (and 1e-8 around iteration 40), although M is
  symmetric to 4e-16 and the preconditioned spectrum lies in [0.17, 5.5];
  perturbations of 1e-16 and 1e-15 give about the same spread, so it is
  the noise of FP64 rounding itself, not a response proportional to eps.

The GPU parity test of the CG iterate (tests/test_gpu_parity.py) therefore
compares at 1e-10 at iterations 15 and 25 and, at the converged count,
against ten times this spread, computed for the same right-hand side with
eps = twice the measured GPU-oracle apply difference (about 2e-15 of the
apply's max-norm: FP64 rounding level, where the spread is flat in eps).
"""
import numpy as np
import pytest

from paper_2304_04876_amd import problems as P
from oracle import gdsw_oracle as O


class PerturbedApply:
    """The oracle's apply with every entry of the result multiplied by
    1 + eps * u, u uniform(-1, 1) from a seeded generator."""

    def __init__(self, M, eps, seed):
        self.M = M
        self.eps = eps
        self.rng = np.random.default_rng(seed)

    def apply(self, r):
        z = self.M.apply(r)
        return z * (1.0 + self.eps * self.rng.uniform(-1.0, 1.0, z.size))


def iterate_spread(A, b, M, k, eps, seeds=(100, 101, 102)):
    """Largest relative 2-norm distance between the k-th CG iterate with the
    exact oracle apply and with perturbed applies."""
    x = O.pcg(A, b, M, fixed_iters=k).x
    worst = 0.0
    for s in seeds:
        y = O.pcg(A, b, PerturbedApply(M, eps, s), fixed_iters=k).x
        worst = max(worst, float(np.linalg.norm(y - x) / np.linalg.norm(x)))
    return worst


@pytest.fixture(scope="module")
def small():
    pr = P.workload_poisson_small()
    return pr, {loc: O.GDSW(pr.A, pr.part, 1, pr.n_parts, local=loc) for loc in ("exact", "ilu0")}


def test_exact_local_solves_keep_iterates_stable(small):
    pr, Ms = small
    b = P.rhs_uniform(pr.n, 0)
    k = O.pcg(pr.A, b, Ms["exact"], rtol=1e-8).iters
    assert iterate_spread(pr.A, b, Ms["exact"], k, 1e-16) <= 1e-14


def test_ilu0_jacobi_iterates_amplify_rounding(small):
    pr, Ms = small
    M = Ms["ilu0"]
    b = P.rhs_uniform(pr.n, 0)
    k = O.pcg(pr.A, b, M, rtol=1e-8).iters
    assert k == 43
    # the operator itself is symmetric to rounding
    r1, r2 = P.rhs_uniform(pr.n, 5), P.rhs_uniform(pr.n, 6)
    a, c = r2 @ M.apply(r1), r1 @ M.apply(r2)
    assert abs(a - c) <= 1e-14 * abs(a)
    early = iterate_spread(pr.A, b, M, 15, 1e-16)
    mid = iterate_spread(pr.A, b, M, 30, 1e-16)
    late = iterate_spread(pr.A, b, M, k, 1e-16)
    # stable early, then growth by orders of magnitude
    assert early <= 1e-14
    assert mid >= 100 * early
    assert 1e-12 <= late <= 1e-9


def test_spread_is_rounding_noise(small):
    """The late spread does not follow the perturbation's size: 1e-15 moves
    the iterate about as much as 1e-16 (both at the level of the oracle's own
    rounding), so any two FP64 evaluations of the operator that differ at
    rounding level give iterates this far apart.  Up to iteration 25 the
    spread stays below 1e-11."""
    pr, Ms = small
    for seed in (0, 1):
        b = P.rhs_uniform(pr.n, seed)
        assert iterate_spread(pr.A, b, Ms["ilu0"], 25, 1e-15) <= 1e-11
        s1 = iterate_spread(pr.A, b, Ms["ilu0"], 35, 1e-16)
        s10 = iterate_spread(pr.A, b, Ms["ilu0"], 35, 1e-15)
        assert 0.2 <= s10 / s1 <= 10.0

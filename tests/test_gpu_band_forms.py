"""The launch forms of the band solves (Sec. V-B, the triangular solves of
the exact local solver after a banded Cholesky factorization) give the same
bits, through the C ABI.  The 1024-thread one-launch form issues each block
step's band loads during the step before; the 256- and 512-thread forms and
the persistent forms load them in the step itself; every sum is formed in
the same order in all of them.

Cases chosen for the paths of the look-ahead form: triangles solved by
substitution (bands narrower than 63), bands wider than the rows it holds
ahead (256 rows below a block in FP64, 384 in FP32), and a band wider than
the workgroup (columns past the first 1024 in the backward pass).  FP64
applies also match the oracle within 1e-12 of its max-norm (two
backward-stable FP64 factorizations of the same well-conditioned matrices)."""
import sys

import numpy as np
import pytest

from paper_2304_04876_amd import binding as B
from paper_2304_04876_amd import problems as P
from oracle import gdsw_oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    # 4^3 boxes: bands of 32 (substitution in the triangles)
    "narrow_band": (lambda: P.poisson3d(12, 3), 0, 62),
    # 20^3 boxes: bands of 440, past the rows held ahead
    "wide_band": (lambda: P.poisson3d(40, 2), 385, 1024),
    # 34 x 34 x 8.5 slabs: bands of 1,156, wider than the workgroup (the
    # band Cholesky's LDS holds bands up to 1,187)
    "band_wider_than_workgroup": (lambda: P.poisson3d(34, (1, 1, 4)), 1025, 1187),
}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("prec", [B.FP64, B.FP32])
@pytest.mark.parametrize("case", list(CASES))
def test_band_launch_forms_bitwise(case, prec):
    make, bmin, bmax = CASES[case]
    pr = make()
    say(f"[band forms] {case} prec={prec} n={pr.n}")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, local=B.LOCAL_EXACT, exact_order=B.ORDER_NATURAL, local_prec=prec,
               basis_prec=B.FP64 if prec == B.FP64 else B.FP32)
    bw = g.info()["max_bandwidth"]
    assert bmin <= bw <= bmax, bw
    r_h = P.rhs_uniform(pr.n, 7)
    r = torch.from_numpy(r_h).cuda()
    first = None
    for v in range(6):
        B.gdsw_set_launch(g.h, v, 0, 1, 0)
        z = torch.zeros_like(r)
        g.apply(r, z)
        if first is None:
            first = z
        assert torch.equal(z, first), v
    if prec == B.FP64:
        M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local="exact")
        zo = M.apply(r_h)
        torch.cuda.synchronize()
        assert np.abs(first.cpu().numpy() - zo).max() <= 1e-12 * np.abs(zo).max()
    g.close()

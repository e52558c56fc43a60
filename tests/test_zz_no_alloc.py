"""The allocation-free apply (gdsw_apply_static, for callers that cannot
allocate device memory): through the C ABI its result equals gdsw_apply's
bit for bit -- same kernels, same order of operations, only the scratch
comes from the library's static device array -- on consecutive calls whose
sizes shrink (stale contents of the shared array must not matter), with the
launch forms that use extra scratch (sweep iterates in global memory, the
blocked coarse prolongation, the coarse chain on a second stream); a handle
that needs more scratch than the array holds is refused with BUDGET."""
import sys

import numpy as np
import pytest

from paper_2304_04876_amd import binding as B
from paper_2304_04876_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(g, seed):
    r = torch.from_numpy(P.rhs_uniform(g.n, seed)).cuda()
    z_ref = torch.zeros_like(r)
    z_st = torch.full_like(r, float("nan"))
    g.apply(r, z_ref)
    B.gdsw_apply_static(g.h, r, z_st)
    torch.cuda.synchronize()
    return z_ref, z_st


def test_static_apply_equals_apply_on_shrinking_calls():
    # 1) large subdomains (iterates of the sweeps in global scratch)
    say("[no-alloc] poisson 40^3, 2^3 boxes, ILU(0) FP64 (streaming sweeps)")
    pa = P.poisson3d(40, 2)
    ga = B.Gdsw(pa.A, pa.part, pa.n_parts, 1, local=B.LOCAL_ILU0)
    # 2) smaller: exact local solves, blocked coarse prolongation, coarse
    #    chain on the second stream
    say("[no-alloc] poisson 16^3, 2^3 boxes, exact, split prolongation, two streams")
    pb = P.poisson3d(16, 2)
    gb = B.Gdsw(pb.A, pb.part, pb.n_parts, 1, local=B.LOCAL_EXACT)
    B.gdsw_set_launch(gb.h, apply_streams=2, prolong_variant=1)
    # 3) smaller still: elasticity, three dofs per node, FP32 factors
    say("[no-alloc] elasticity 4^3, 2^3 boxes, FP32 band factors")
    pc = P.elasticity_q1(4, 2)
    gc = B.Gdsw(pc.A, pc.part, pc.n_parts, 3, P.rigid_body_modes(pc), local=B.LOCAL_EXACT,
                local_prec=B.FP32, basis_prec=B.FP32)
    for name, g, seed in (("40^3", ga, 1), ("16^3", gb, 2), ("elasticity 4^3", gc, 3), ("40^3 again", ga, 4)):
        z_ref, z_st = _pair(g, seed)
        say(f"  {name}: n={g.n} equal={bool(torch.equal(z_ref, z_st))}")
        assert torch.equal(z_ref, z_st), name
        assert float(z_ref.abs().max()) > 0
    # queued back to back on one stream, different handles, no host sync
    r1 = torch.from_numpy(P.rhs_uniform(ga.n, 7)).cuda()
    r2 = torch.from_numpy(P.rhs_uniform(gb.n, 8)).cuda()
    z1, z2 = torch.zeros_like(r1), torch.zeros_like(r2)
    B.gdsw_apply_static(ga.h, r1, z1)
    B.gdsw_apply_static(gb.h, r2, z2)
    e1, e2 = torch.zeros_like(r1), torch.zeros_like(r2)
    ga.apply(r1, e1)
    gb.apply(r2, e2)
    torch.cuda.synchronize()
    assert torch.equal(z1, e1) and torch.equal(z2, e2)
    for g in (ga, gb, gc):
        g.close()


def test_static_apply_refuses_a_handle_beyond_the_array():
    # 8 x 8 x 4 boxes of 16 x 16 x 32 nodes (up to 10,752 rows each with the
    # overlap, 2,654,208 in all): the ILU(0) FP64 sweep iterates live in
    # global scratch, 24 B per local row (63.7 MB), beside the local results
    # (21.2 MB): more than the 64 MiB array
    say("[no-alloc] poisson 128^3, 8x8x4 boxes, ILU(0) FP64: beyond the static array")
    pr = P.poisson3d(128, (8, 8, 4))
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, local=B.LOCAL_ILU0)
    r = torch.from_numpy(P.rhs_uniform(g.n, 0)).cuda()
    z = torch.zeros_like(r)
    with pytest.raises(B.GdswError) as ei:
        B.gdsw_apply_static(g.h, r, z)
    assert ei.value.status == 5 and "static array" in str(ei.value)
    # the handle itself is unaffected
    g.apply(r, z)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(z).all())
    g.close()

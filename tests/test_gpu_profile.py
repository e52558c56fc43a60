"""Timing of the local solves inside applies (gdsw_profile_local /
gdsw_profile_read; Sec. VII times the local-solver phase on its own): one
record per apply that runs the local solves, none under graph capture,
positive durations, and results unchanged by the recording."""
import sys

import numpy as np
import pytest

from paper_2304_04876_amd import binding as B
from paper_2304_04876_amd import problems as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_profile_records_local_solves():
    pr = P.poisson3d(16, 2)
    say("[profile] poisson16 ilu0")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, local=B.LOCAL_ILU0)
    r = torch.from_numpy(P.rhs_uniform(pr.n, 5)).cuda()
    z0 = torch.zeros_like(r)
    g.apply(r, z0)
    B.gdsw_profile_local(g.h, True)
    z = torch.zeros_like(r)
    for _ in range(3):
        g.apply(r, z)
        torch.cuda.synchronize()
        assert torch.equal(z, z0)
    g.apply_part(r, z, 2)          # coarse part only: no local solve, no record
    g.apply_part(r, z, 1)          # one-level part: recorded
    d = B.gdsw_profile_read(g.h)
    assert d.size == 4 and np.all(d > 0), d
    # nothing is recorded while the stream is captured
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g.apply(r, z)
    torch.cuda.synchronize()
    n_before = B.gdsw_profile_read(g.h).size
    assert n_before == 5
    with torch.cuda.graph(graph):
        B.gdsw_apply(g.h, r, z, torch.cuda.current_stream())
    torch.cuda.synchronize()
    z.zero_()
    graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(z, z0)
    assert B.gdsw_profile_read(g.h).size == n_before
    # a CG solve records one local solve per apply it runs
    B.gdsw_profile_local(g.h, True)    # clears
    x = torch.zeros_like(r)
    out = g.solve(r, x, rtol=1e-8)
    d = B.gdsw_profile_read(g.h)
    assert d.size >= out["iterations"] + 1
    # stopping keeps the records; later applies are not recorded
    B.gdsw_profile_local(g.h, False)
    g.apply(r, z)
    assert B.gdsw_profile_read(g.h).size == d.size
    g.close()

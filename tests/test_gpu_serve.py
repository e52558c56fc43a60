"""The serving loop: resident operators, continuous batching of requests that
arrive while others run, and each result identical alone and in the mix."""
import os
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_2304_04876_amd import binding as B
from paper_2304_04876_amd import problems as P
from paper_2304_04876_amd import serve as SV

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_served_results_equal_alone():
    print("[serve] 3 operators, 2 slots each, 24 requests", file=sys.stderr, flush=True)
    ops = [P.poisson3d(12, 2), P.poisson3d(16, 2), P.poisson3d(10, 1)]
    srv = SV.Server(ops, slots_per_op=2, local=B.LOCAL_ILU0, local_prec=B.FP16, basis_prec=B.FP32,
                    step_iters=2)
    t, opi = SV.poisson_arrivals(24, 400.0, len(ops), seed=3)
    reqs = [SV.Request(rid=i, op=int(opi[i]), arrival=float(t[i]), b=P.rhs_uniform(ops[int(opi[i])].n, 100 + i))
            for i in range(24)]
    reqs, sols = srv.run(reqs, keep_solutions=True)
    srv.close()
    # requests overlapped on the device: some started while others ran
    overlap = sum(1 for a in reqs for b in reqs if a.rid < b.rid and b.start < a.finish and a.start < b.finish)
    assert overlap > 0
    alone = [B.Gdsw(op.A, op.part, op.n_parts, 1, local=B.LOCAL_ILU0, local_prec=B.FP16, basis_prec=B.FP32)
             for op in ops]
    for r in reqs:
        assert r.status == 0 and r.rel_res_true <= 1.5e-8
        bd = torch.from_numpy(r.b).cuda()
        xd = torch.zeros_like(bd)
        out = alone[r.op].solve(bd, xd, rtol=1e-8)
        assert out["iterations"] == r.iterations
        assert torch.equal(xd, sols[r.rid]), r.rid
        # and the solution is the FP64 one to the accuracy the tolerance allows
        x = spla.spsolve(ops[r.op].A.tocsc(), r.b)
        assert np.linalg.norm(sols[r.rid].cpu().numpy() - x) <= 1e-6 * np.linalg.norm(x)
    for g in alone:
        g.close()


def test_budget_admission():
    ops = [P.poisson3d(10, 2), P.poisson3d(12, 2)]
    probe = SV.Server(ops, slots_per_op=1, local=B.LOCAL_ILU0, local_prec=B.FP16, basis_prec=B.FP32)
    resident, per_slot = probe.operator_bytes, probe.slot_workspace_bytes
    one = probe.device_bytes
    probe.close()
    # the operators are held once, each slot adds only its workspace
    assert 0 < per_slot < resident
    assert one == resident + per_slot
    # a budget for the operators and two and a half slot workspaces
    srv = SV.Server(ops, hbm_budget_bytes=int(resident + 2.5 * per_slot), local=B.LOCAL_ILU0,
                    local_prec=B.FP16, basis_prec=B.FP32)
    assert srv.slots_per_op == 2
    assert srv.device_bytes == resident + 2 * per_slot
    srv.close()
    with pytest.raises(B.GdswError):
        SV.Server(ops, hbm_budget_bytes=1000, local=B.LOCAL_ILU0)


GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_serve_oracle.npz")


@pytest.mark.parametrize("prec", [B.FP64, B.FP16])
def test_served_results_against_oracle(prec):
    """Three operators of the serving stream (Poisson N = 32, 59, 96 with
    P = round(N/16), ILU(0) + 5+5 Jacobi sweeps, GDSW), one request each,
    served together: FP64 local factors reproduce the oracle's iteration
    counts; with the stream's FP16 factors (FP32 arithmetic) the iteration
    counts stay within the reduced-precision slack and each result's error
    against the FP64 oracle's solution is stated and bounded by what two
    solutions with relative residuals <= 1e-8 can differ by."""
    ref = np.load(GOLD)
    Ns = [int(v) for v in ref["serve_N"]]
    ops = [P.serve_operator(N) for N in Ns]
    print(f"[serve] oracle samples N={Ns} prec={prec}", file=sys.stderr, flush=True)
    srv = SV.Server(ops, slots_per_op=1, local=B.LOCAL_ILU0, local_prec=prec,
                    basis_prec=B.FP64 if prec == B.FP64 else B.FP32, step_iters=4)
    reqs = [SV.Request(rid=int(ref["serve_rid"][j]), op=j, arrival=0.0,
                       b=P.rhs_uniform(ops[j].n, int(ref["serve_rid"][j]))) for j in range(len(ops))]
    reqs, sols = srv.run(reqs, keep_solutions=True)
    srv.close()
    for j, r in enumerate(sorted(reqs, key=lambda q: q.op)):
        N = Ns[r.op]
        xs = sols[r.rid].cpu().numpy()[ref["serve_idx"][r.op]]
        err = np.abs(xs - ref["serve_x"][r.op]).max() / float(ref["serve_x_norm2"][r.op])
        oit = int(ref["serve_iters"][r.op])
        print(f"  N={N}: iterations {r.iterations} (oracle {oit}), solution diff vs the FP64 oracle "
              f"{err:.1e} of its 2-norm", file=sys.stderr, flush=True)
        assert r.status == 0 and r.rel_res_true <= 1.5e-8
        assert abs(r.iterations - oit) <= (1 if prec == B.FP64 else 4)
        # true residuals <= 1.5e-8 ||b|| here and about 1e-8 ||b|| in the
        # oracle: ||x - x_oracle|| <= 3e-8 ||A^-1|| ||b||, with
        # ||A^-1|| = 1 / (12 sin^2(pi / (2 (N + 1)))) for this stencil
        lam_min = 12.0 * np.sin(np.pi / (2 * (N + 1))) ** 2
        bound = 3e-8 * np.linalg.norm(r.b) / lam_min / float(ref["serve_x_norm2"][r.op])
        assert err <= bound, (N, err, bound)

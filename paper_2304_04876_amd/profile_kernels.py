"""Launches the kernels whose hardware counters are reported, for use under
rocprofv3 (kernel trace, FETCH_SIZE / WRITE_SIZE passes):

* the batched local-solve kernel of the 128^3 Poisson workload (512
  subdomains, ILU(0) + 5+5 Jacobi sweeps or banded Cholesky), or with
  ``--elasticity`` of the Q1 elasticity workload (48^3 elements, 6^3
  boxes, banded Cholesky), ``--reps`` times;
* the full preconditioner apply once;
* a plain device copy of a known size (``--copy-mib`` MiB read and written),
  ``--reps`` times, to calibrate the byte counters;
* with ``--setup-only``, only the numerical setup (band Cholesky, inverted
  diagonal blocks, extension, coarse matrix and its Gauss-Jordan inverse),
  for the arithmetic counters of the dense setup kernels.

Usage: python -m paper_2304_04876_amd.profile_kernels [--local ilu0|exact]
"""
from __future__ import annotations

import argparse
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--local", choices=["ilu0", "exact"], default="ilu0")
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16", "fp16"], default="fp64")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--P", type=int, default=8)
    ap.add_argument("--elasticity", action="store_true")
    ap.add_argument("--ilu-level", type=int, default=0)
    ap.add_argument("--factor-sweeps", type=int, default=0)
    ap.add_argument("--exact-order", choices=["natural", "nd", "auto"], default="natural",
                    help="exact local solves: band (natural order), supernodal after nested dissection, "
                         "or per subdomain the one with fewer factor values")
    ap.add_argument("--tune", action="store_true", help="autotune the launch configurations first "
                    "(as the benchmark does), so the counters see the configuration it times")
    ap.add_argument("--setup-only", action="store_true", help="only the numerical setup (local factors, "
                    "extension, coarse matrix and its inverse), for counters of the setup kernels")
    a = ap.parse_args()

    import torch
    from paper_2304_04876_amd import binding as B
    from paper_2304_04876_amd import problems as P

    precs = {"fp64": B.FP64, "fp32": B.FP32, "bf16": B.BF16, "fp16": B.FP16}
    if a.elasticity:
        pr = P.workload_elasticity()
        Z = P.rigid_body_modes(pr)
    else:
        pr = P.poisson3d(a.N, a.P)
        Z = None
    print(f"[profile] setup {pr.name} local={a.local} order={a.exact_order} prec={a.prec}", file=sys.stderr,
          flush=True)
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, pr.dpn, Z,
               local=B.LOCAL_ILU0 if a.local == "ilu0" else B.LOCAL_EXACT, local_prec=precs[a.prec],
               basis_prec=B.FP64 if a.prec == "fp64" else B.FP32, ilu_level=a.ilu_level,
               ilu_factor_sweeps=a.factor_sweeps,
               exact_order={"natural": B.ORDER_NATURAL, "nd": B.ORDER_ND, "auto": B.ORDER_AUTO}[a.exact_order])
    torch.cuda.synchronize()
    if a.setup_only:
        g.close()
        print("[profile] done", file=sys.stderr, flush=True)
        return
    r = torch.from_numpy(P.rhs_uniform(pr.n, 0)).cuda()
    z = torch.zeros_like(r)
    torch.cuda.synchronize()
    if a.tune:
        times = B.gdsw_autotune(g.h, reps=3)
        print(f"[profile] autotune {times} -> local variant {g.info()['local_variant']}", file=sys.stderr,
              flush=True)
    print(f"[profile] local solves x{a.reps}", file=sys.stderr, flush=True)
    for _ in range(a.reps):
        g.apply_part(r, None, 4)
    g.apply(r, z)
    torch.cuda.synchronize()
    n = a.copy_mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    print(f"[profile] copy {a.copy_mib} MiB x{a.reps}", file=sys.stderr, flush=True)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    g.close()
    print("[profile] done", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()

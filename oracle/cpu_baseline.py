"""CPU baseline of the benchmark: the FP64 oracle timed on the host cores
(TEST INFRASTRUCTURE ONLY; run as a child process of the benchmark, before
or apart from any GPU work, so that it never shares a process with a GPU
context).

    python -m oracle.cpu_baseline --workload poisson --N 128 --P 8 --local ilu0 --seed 2

Sets up the oracle for the workload (untimed), then times one full solve of
the right-hand side with BLAS limited to one thread: once with the serial
subdomain loop (1 core) and once with the loop spread over ``--workers``
processes (default: the cores this process may run on, at most 16).  Prints
one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["poisson", "elasticity"], default="poisson")
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--P", type=int, default=8)
    ap.add_argument("--local", choices=["ilu0", "exact"], default="ilu0")
    ap.add_argument("--coarse", choices=["gdsw", "rgdsw"], default="gdsw")
    ap.add_argument("--gmres", choices=["single_reduce", "classical"], default="single_reduce")
    ap.add_argument("--ilu-level", type=int, default=0)
    ap.add_argument("--factor-sweeps", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0, help="right-hand side seed (Poisson)")
    ap.add_argument("--scale", type=float, default=1.0, help="load scale (elasticity)")
    ap.add_argument("--workers", type=int, default=0)
    args = ap.parse_args()

    from threadpoolctl import threadpool_limits
    from paper_2304_04876_amd import problems as P
    from oracle import gdsw_oracle as O
    from oracle.parallel import ForkedApply

    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = args.workers or min(avail, 16)
    elastic = args.workload == "elasticity"
    if elastic:
        pr = P.elasticity_q1(args.N, args.P)
        Z = P.rigid_body_modes(pr)
        b = pr.b * args.scale
    else:
        pr = P.poisson3d(args.N, args.P)
        Z = None
        b = P.rhs_uniform(pr.n, args.seed)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        M = O.GDSW(pr.A, pr.part, pr.dpn, pr.n_parts, Z=Z, local=args.local, ilu_level=args.ilu_level,
                   factor_sweeps=args.factor_sweeps, coarse_space=args.coarse)
        t_setup = time.perf_counter() - t0

        def solve(Mx):
            if elastic:
                f = O.gmres_single_reduce if args.gmres == "single_reduce" else O.gmres
                return f(pr.A, b, Mx, rtol=1e-8, restart=30)
            return O.pcg(pr.A, b, Mx, rtol=1e-8)

        t0 = time.perf_counter()
        res1 = solve(M)
        t1 = time.perf_counter() - t0
        with ForkedApply(M, workers) as F:
            t0 = time.perf_counter()
            resw = solve(F)
            tw = time.perf_counter() - t0
            used = F.workers
    assert resw.iters == res1.iters
    print(json.dumps({
        "setup_s": round(t_setup, 2), "iterations": int(res1.iters),
        "serial_s": round(t1, 3), "serial_solves_per_s": round(1.0 / t1, 5),
        "parallel_s": round(tw, 3), "parallel_solves_per_s": round(1.0 / tw, 5),
        "workers": int(used), "cores_available": int(avail), "nproc": os.cpu_count(),
        "cpu_model": cpu_model(), "rel_res_true": float(res1.rel_res_true),
    }), flush=True)


if __name__ == "__main__":
    main()

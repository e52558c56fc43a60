"""Writes batch_serve_oracle.npz: FP64 oracle results, sampled, for the
parity tests of the batched and the served workloads.

Calls only the oracle and the seeded input generators.

Batch (256 diffusion problems from batch_diffusion_specs(256); exact local
solves, GDSW): eight problems chosen by a fixed rule so that the grid edge
spans [16, 48] and every box count P in {2, 3, 4} appears -- for each P the
problems with the smallest and the largest N, then the two problems of
median N among the rest.  Stored per chosen problem j (arrays stacked, ragged
ones padded with -1 / 0):
  batch_k[j]        index of the problem in the batch
  batch_idx[j]      512 sampled local dof indices (seed 100 + k)
  batch_z[j]        (M^{-1} b_k)[idx], b_k the problem's right-hand side
  batch_z_norm[j]   max |M^{-1} b_k|
  batch_iters[j]    CG iterations to 1e-8
  batch_x[j]        the CG solution at idx, batch_x_norm[j] its max-norm,
                    batch_x_norm2[j] its 2-norm
  batch_xf[j]       the CG iterate after exactly batch_iters[j] iterations

Serving (Poisson operators N = 32, 59, 96 with P = round(N/16); ILU(0) local
solves with 5+5 Jacobi sweeps in FP64, GDSW): one request each, right-hand
side rhs_uniform(n, rid) with rid = 1000, 1001, 1002:
  serve_N[j], serve_rid[j], serve_idx[j] (512 samples, seed 200 + j),
  serve_iters[j], serve_x[j] (CG solution to 1e-8 at idx),
  serve_x_norm[j] (max-norm), serve_x_norm2[j] (2-norm)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2304_04876_amd import problems as P  # noqa: E402
from oracle import gdsw_oracle as O  # noqa: E402

NS = 512


def chosen_batch_problems(specs):
    """The fixed selection rule of the module docstring."""
    pick = []
    for Pn in (2, 3, 4):
        cand = [s for s in specs if s["P"] == Pn]
        cand.sort(key=lambda s: (s["N"], s["k"]))
        for s in (cand[0], cand[-1]):
            if s["k"] not in pick:
                pick.append(s["k"])
    rest = sorted([s for s in specs if s["k"] not in pick], key=lambda s: (s["N"], s["k"]))
    mid = len(rest) // 2
    for s in rest[mid - 1:mid + 1]:
        pick.append(s["k"])
    return pick


def main():
    specs = P.batch_diffusion_specs(256)
    ks = chosen_batch_problems(specs)
    out = {k: [] for k in ("batch_k", "batch_idx", "batch_z", "batch_z_norm", "batch_iters", "batch_x",
                           "batch_x_norm", "batch_x_norm2", "batch_xf")}
    for k in ks:
        t = time.time()
        pr = P.batch_diffusion_problem(specs[k])
        M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local="exact")
        idx = np.sort(np.random.default_rng(100 + k).choice(pr.n, NS, replace=False))
        z = M.apply(pr.b)
        res = O.pcg(pr.A, pr.b, M, rtol=1e-8)
        fx = O.pcg(pr.A, pr.b, M, fixed_iters=res.iters)
        out["batch_k"].append(k)
        out["batch_idx"].append(idx)
        out["batch_z"].append(z[idx])
        out["batch_z_norm"].append(np.abs(z).max())
        out["batch_iters"].append(res.iters)
        out["batch_x"].append(res.x[idx])
        out["batch_x_norm"].append(np.abs(res.x).max())
        out["batch_x_norm2"].append(np.linalg.norm(res.x))
        out["batch_xf"].append(fx.x[idx])
        print(f"batch problem {k}: N={specs[k]['N']} P={specs[k]['P']} iters={res.iters} "
              f"({time.time() - t:.1f} s)", flush=True)
    sv = {k: [] for k in ("serve_N", "serve_rid", "serve_idx", "serve_iters", "serve_x", "serve_x_norm", "serve_x_norm2")}
    for j, (N, rid) in enumerate(((32, 1000), (59, 1001), (96, 1002))):
        t = time.time()
        pr = P.serve_operator(N)
        M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local="ilu0", sweeps=5)
        b = P.rhs_uniform(pr.n, rid)
        res = O.pcg(pr.A, b, M, rtol=1e-8)
        idx = np.sort(np.random.default_rng(200 + j).choice(pr.n, NS, replace=False))
        sv["serve_N"].append(N)
        sv["serve_rid"].append(rid)
        sv["serve_idx"].append(idx)
        sv["serve_iters"].append(res.iters)
        sv["serve_x"].append(res.x[idx])
        sv["serve_x_norm"].append(np.abs(res.x).max())
        sv["serve_x_norm2"].append(np.linalg.norm(res.x))
        print(f"serve N={N} rid={rid}: iters={res.iters} ({time.time() - t:.1f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "batch_serve_oracle.npz"),
                        **{k: np.array(v) for k, v in out.items()}, **{k: np.array(v) for k, v in sv.items()})


if __name__ == "__main__":
    main()

"""Writes large_poisson_oracle.npz: the FP64 oracle's results on the 128^3
Poisson workload with 512 boxes (ILU(0) local solves with 5+5 Jacobi sweeps,
GDSW coarse space), sampled, for the full-size GPU parity test; with the
argument `exact`, large_poisson_exact_oracle.npz: the same with exact local
solves (same sample indices and fields, z_exact in place of z_ilu0).

Calls only the oracle and the seeded input generators.  Stored:
  idx       4096 sampled dof indices (fixed seed 7)
  z_ilu0    (M^{-1} r)[idx] for r = rhs_uniform(n, 0)
  zc        coarse term (Phi A0^{-1} Phi^T r)[idx]
  cg_iters  oracle CG iterations to 1e-8 for seeds 0 and 1
  x_fixed   CG iterate after cg_iters[0] iterations, seed 0, at idx
  a0_diag   diagonal of A0; a0_samp rows/cols/values of 2000 sampled entries
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2304_04876_amd import problems as P  # noqa: E402
from oracle import gdsw_oracle as O  # noqa: E402


def main():
    local = sys.argv[1] if len(sys.argv) > 1 else "ilu0"
    pr = P.workload_poisson_large()
    t = time.time()
    M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local=local, sweeps=5)
    print("oracle setup", time.time() - t, flush=True)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(pr.n, 4096, replace=False))
    r = P.rhs_uniform(pr.n, 0)
    z = M.apply(r)
    zc = M.coarse_apply(r)
    its = []
    for seed in (0, 1):
        res = O.pcg(pr.A, P.rhs_uniform(pr.n, seed), M, rtol=1e-8)
        its.append(res.iters)
        print("seed", seed, "iters", res.iters, flush=True)
    fx = O.pcg(pr.A, r, M, fixed_iters=its[0])
    n0 = M.A0.shape[0]
    ar = rng.integers(0, n0, 2000)
    ac = rng.integers(0, n0, 2000)
    name = "large_poisson_oracle.npz" if local == "ilu0" else f"large_poisson_{local}_oracle.npz"
    np.savez_compressed(os.path.join(HERE, name), idx=idx, **{f"z_{local}": z[idx]}, zc=zc[idx],
                        cg_iters=np.array(its), x_fixed=fx.x[idx], a0_diag=np.diag(M.A0).copy(),
                        a0_rows=ar, a0_cols=ac, a0_vals=M.A0[ar, ac], z_norm=np.abs(z).max(),
                        x_norm=np.linalg.norm(fx.x))


if __name__ == "__main__":
    main()

"""Writes elasticity_oracle.npz (GDSW coarse space) or, with the argument
`rgdsw`, elasticity_rgdsw_oracle.npz (the reduced GDSW space): the FP64
oracle on the Q1 elasticity workload (48^3 elements, 6^3 boxes, 6 rigid-body
modes, exact local solves), sampled, for the full-size GPU parity test.

Calls only the oracle and the seeded input generators.  Stored:
  idx       4096 sampled dof indices (seed 11)
  z         (M^{-1} b)[idx] for the assembled load b
  n0        coarse dimension
  a0_diag   diagonal of A0
  gm_iters  right-preconditioned GMRES(30) iterations to 1e-8
  x_gm      the GMRES solution at idx
  x_fixed   the GMRES(30) iterate after exactly gm_iters iterations at idx
            (modified Gram-Schmidt Arnoldi), and its 2-norm x_fixed_norm
  sr_iters, x_fixed_sr
            the single-reduce GMRES(30): iterations to 1e-8 and the iterate
            after exactly sr_iters iterations at idx
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
    coarse = sys.argv[1] if len(sys.argv) > 1 else "gdsw"
    pr = P.workload_elasticity()
    Z = P.rigid_body_modes(pr)
    t = time.time()
    M = O.GDSW(pr.A, pr.part, 3, pr.n_parts, Z=Z, local="exact", coarse_space=coarse)
    print("oracle setup", time.time() - t, flush=True)
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(pr.n, 4096, replace=False))
    z = M.apply(pr.b)
    t = time.time()
    res = O.gmres(pr.A, pr.b, M, rtol=1e-8, restart=30)
    print("gmres", res.iters, time.time() - t, flush=True)
    fx = O.gmres(pr.A, pr.b, M, restart=30, fixed_iters=res.iters)
    sr = O.gmres_single_reduce(pr.A, pr.b, M, rtol=1e-8, restart=30)
    fsr = O.gmres_single_reduce(pr.A, pr.b, M, restart=30, fixed_iters=sr.iters)
    print("single-reduce gmres", sr.iters, flush=True)
    name = "elasticity_oracle.npz" if coarse == "gdsw" else f"elasticity_{coarse}_oracle.npz"
    np.savez_compressed(os.path.join(HERE, name), idx=idx, z=z[idx], z_norm=np.abs(z).max(),
                        n0=M.A0.shape[0], a0_diag=np.diag(M.A0).copy(), gm_iters=res.iters, x_gm=res.x[idx],
                        x_norm=np.abs(res.x).max(), x_fixed=fx.x[idx], x_fixed_norm=np.abs(fx.x).max(),
                        sr_iters=sr.iters, x_fixed_sr=fsr.x[idx])


if __name__ == "__main__":
    main()

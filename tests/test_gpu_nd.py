"""GPU parity of the nested-dissection supernodal exact local solver
(options.exact_order = ND or AUTO; Sec. V-B, the sparse direct factorization
of each A_i after a fill-reducing ordering) against the FP64 oracle, which
factors the same A_i by a sparse LU, through the C ABI.

Tolerances: the apply within 1e-12 of the oracle's max-norm, as for the
banded exact solver (two backward-stable FP64 factorizations of the same
well-conditioned local matrices, condition numbers below 1e4 here); CG
iteration counts within +-1 of the oracle's.  Bitwise: results do not depend
on the launch configuration, on the slot a right-hand side sits in, on what
a problem is packed with, or on the allocation-free entry point (the
solve's lanes per item depend on the subdomain alone)."""
import sys

import numpy as np
import pytest

from paper_2304_04876_amd import binding as B
from paper_2304_04876_amd import problems as P
from oracle import gdsw_oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ND = dict(local=B.LOCAL_EXACT, exact_order=B.ORDER_ND)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = {
    "poisson20_P2": lambda: (P.poisson3d(20, 2), None),
    "poisson12_P3": lambda: (P.poisson3d(12, 3), None),
    "poisson17_P3_ragged": lambda: (P.poisson3d(17, 3), None),
    "poisson10_P231": lambda: (P.poisson3d(10, (2, 3, 1)), None),
    "diffusion20_P3": lambda: (P.diffusion3d(20, np.exp(np.random.default_rng(9).standard_normal(21 ** 3)), 3),
                               None),
    # 12,100-row subdomains: too large for LDS with FP64 factors, they keep the band
    "diffusion_large_subdomains": lambda: (P.batch_diffusion_problem(P.batch_diffusion_specs(2)[1]), None),
    "elasticity6_P2": lambda: ((lambda p: (p, P.rigid_body_modes(p)))(P.elasticity_q1(6, 2))),
}


@pytest.mark.parametrize("case", list(CASES))
def test_nd_apply_matches_oracle(case):
    pr, Z = CASES[case]()
    say(f"[nd] apply {case} n={pr.n}")
    M = O.GDSW(pr.A, pr.part, pr.dpn, pr.n_parts, Z=Z, local="exact")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, pr.dpn, Z, **ND)
    # every nonempty subdomain whose FP64 solve fits 160 KiB of LDS (at most
    # 10,648 rows; these subdomains have far fewer than 2,048 supernodes and
    # 2,048 rows of one height above the leaves)
    ni = np.diff(B.gdsw_copy_map(g.h, B.MAP_OV_PTR))
    fits = int(((ni > 0) & (ni <= 10648)).sum())
    assert g.info()["nd_subdomains"] == fits
    assert fits > 0 or case == "diffusion_large_subdomains"
    r = P.rhs_uniform(pr.n, 11)
    rd, zd = dev(r), torch.zeros(pr.n, dtype=torch.float64, device="cuda")
    g.apply(rd, zd)
    assert rel_max(host(zd), M.apply(r)) <= 1e-12
    g.apply_part(rd, zd, 1)
    assert rel_max(host(zd), M.apply(r) - M.coarse_apply(r)) <= 1e-12
    g.close()


def test_nd_auto_mixes_band_and_supernodal_subdomains():
    """20^3 in 3^3 boxes: AUTO gives most of the 27 subdomains the
    supernodal factor and keeps the band for the others (20 and 7 with
    leaves of 48 rows); the apply and a CG solve match the oracle."""
    pr = P.poisson3d(20, 3)
    say("[nd] auto mix 20^3")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, local=B.LOCAL_EXACT, exact_order=B.ORDER_AUTO)
    k = g.info()["nd_subdomains"]
    assert 0 < k < pr.n_parts
    M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local="exact")
    r = P.rhs_uniform(pr.n, 4)
    rd = dev(r)
    z = torch.zeros_like(rd)
    g.apply(rd, z)
    assert rel_max(host(z), M.apply(r)) <= 1e-12
    x = torch.zeros_like(rd)
    out = g.solve(rd, x, rtol=1e-8)
    ref = O.pcg(pr.A, r, M, rtol=1e-8)
    assert abs(out["iterations"] - ref.iters) <= 1 and out["rel_res_true"] <= 1.5e-8
    g.close()


def test_nd_launch_configurations_bitwise():
    """Every local-solve launch configuration (the supernodal solves with 256,
    512 and 1024 threads) gives the same bits."""
    pr = P.poisson3d(20, 2)
    say("[nd] launch configurations")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, **ND)
    r = dev(P.rhs_uniform(pr.n, 5))
    first = None
    for v in range(6):
        B.gdsw_set_launch(g.h, v, 0, 1, 0)
        z = torch.zeros_like(r)
        g.apply(r, z)
        if first is None:
            first = z
        assert torch.equal(z, first), v
    g.close()


def test_nd_solve_matches_oracle_and_is_deterministic():
    pr = P.poisson3d(20, 2)
    say("[nd] CG")
    g = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, **ND)
    M = O.GDSW(pr.A, pr.part, 1, pr.n_parts, local="exact")
    b = P.rhs_uniform(pr.n, 0)
    bd = dev(b)
    x1, x2 = torch.zeros_like(bd), torch.zeros_like(bd)
    o1 = g.solve(bd, x1, rtol=1e-8)
    o2 = g.solve(bd, x2, rtol=1e-8)
    ref = O.pcg(pr.A, b, M, rtol=1e-8)
    assert abs(o1["iterations"] - ref.iters) <= 1 and o1["rel_res_true"] <= 1.5e-8
    assert o1["iterations"] == o2["iterations"] and torch.equal(x1, x2)
    g.close()


def test_nd_slots_equal_single_slot():
    """Three right-hand-side slots on one factored operator: each slot's
    apply equals the one-slot handle's, bit for bit."""
    pr = P.poisson3d(16, 2)
    say("[nd] slots")
    g1 = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, **ND)
    g3 = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, slots=3, **ND)
    rs = [dev(P.rhs_uniform(pr.n, 20 + k)) for k in range(3)]
    z3 = torch.zeros(3 * pr.n, dtype=torch.float64, device="cuda")
    g3.apply(torch.cat(rs), z3)
    for k, r in enumerate(rs):
        z = torch.zeros_like(r)
        g1.apply(r, z)
        assert torch.equal(z, z3[k * pr.n:(k + 1) * pr.n]), k
    g1.close()
    g3.close()


def test_nd_batch_equals_alone():
    rng = np.random.default_rng(5)
    probs = [P.diffusion3d(14, np.exp(rng.standard_normal(15 ** 3)), 2),
             P.diffusion3d(11, np.exp(rng.standard_normal(12 ** 3)), 3), P.poisson3d(9, 2)]
    say("[nd] batch vs alone")
    hb = B.gdsw_analyze_batch([(p.A, p.part, p.n_parts) for p in probs], options=B.gdsw_default_options(**ND))
    B.gdsw_factor(hb)
    offs = B.gdsw_problem_offsets(hb)
    r = torch.from_numpy(np.concatenate([P.rhs_uniform(p.n, 10 + k) for k, p in enumerate(probs)])).cuda()
    zb = torch.zeros_like(r)
    B.gdsw_apply(hb, r, zb)
    for k, p in enumerate(probs):
        g = B.Gdsw(p.A, p.part, p.n_parts, 1, **ND)
        rk = r[offs[k]:offs[k + 1]].clone()
        zk = torch.zeros_like(rk)
        g.apply(rk, zk)
        assert torch.equal(zk, zb[offs[k]:offs[k + 1]]), k
        g.close()
    B.gdsw_destroy(hb)


@pytest.mark.parametrize("prec", [B.FP32, B.FP16])
def test_nd_reduced_precision_factors(prec):
    """Supernodal factors stored in FP32 / FP16 (FP32 accumulation): CG meets
    the same tolerance within a few iterations of the FP64 factor."""
    pr = P.poisson3d(16, 2)
    say(f"[nd] precision {prec}")
    g64 = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, **ND)
    glo = B.Gdsw(pr.A, pr.part, pr.n_parts, 1, local_prec=prec, basis_prec=B.FP32, **ND)
    bd = dev(P.rhs_uniform(pr.n, 0))
    x64, xlo = torch.zeros_like(bd), torch.zeros_like(bd)
    o64 = g64.solve(bd, x64, rtol=1e-8)
    olo = glo.solve(bd, xlo, rtol=1e-8)
    assert olo["converged"] and olo["rel_res_true"] <= 2e-8
    assert abs(olo["iterations"] - o64["iterations"]) <= {B.FP32: 1, B.FP16: 4}[prec], (olo, o64)
    g64.close()
    glo.close()


def test_nd_static_apply_and_refactor():
    """The allocation-free apply equals gdsw_apply bit for bit with the
    supernodal solves (their struct products in the static array); a numeric
    re-setup to new coefficients matches a fresh oracle."""
    N, Pn = 14, 3
    k1 = np.exp(np.random.default_rng(71).standard_normal((N + 1) ** 3))
    k2 = np.exp(2.0 * np.random.default_rng(72).standard_normal((N + 1) ** 3))
    p1, p2 = P.diffusion3d(N, k1, Pn), P.diffusion3d(N, k2, Pn)
    say("[nd] static apply, refactor")
    g = B.Gdsw(p1.A, p1.part, p1.n_parts, 1, **ND)
    r = dev(P.rhs_uniform(p1.n, 3))
    z, zs = torch.zeros_like(r), torch.full_like(r, float("nan"))
    g.apply(r, z)
    B.gdsw_apply_static(g.h, r, zs)
    torch.cuda.synchronize()
    assert torch.equal(z, zs)
    B.gdsw_refactor(g.h, p2.A.tocsr().data)
    g.apply(r, z)
    M2 = O.GDSW(p2.A, p2.part, 1, p2.n_parts, local="exact")
    assert rel_max(host(z), M2.apply(host(r))) <= 1e-12
    g.close()

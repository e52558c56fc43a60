"""Throughput benchmark of the GDSW-preconditioned Krylov solves on one MI355X.

Headline workload (``value``): 3D Poisson, 7-point finite differences on the
128^3 interior grid (2,097,152 dofs), 8x8x8 = 512 box subdomains, algebraic
overlap one, GDSW coarse space (2,863 columns), local ILU(0) with 5+5 Jacobi
sweeps, FP64 CG to a relative residual of 1e-8, right-hand sides
uniform(-1, 1) from seeds.  All inputs are synthetic and resident in HBM
before timing.

A step is one complete preconditioned CG solve of a fresh right-hand side
with the factored preconditioner resident (the solve phase of the paper's
three-phase structure); the symbolic analysis and the numerical setup are
timed separately and reported beside it.

The default run prints one JSON line: solves/s (value), applies/s of a
hipGraph-replayed apply, the solve-time p50/p99 of the closed loop, the
roofline of the dominant kernel, the error against FP64 oracle samples, and
sub-records of the other workloads at reduced step counts: the same problem
with exact local solves and with FP16 local factors, Q1 elasticity (FP32
factors, reduced GDSW, single-reduce GMRES(30)), the 256-problem diffusion
batch and the serving stream (latency = completion - arrival); the CPU
baseline is the FP64 oracle timed in a child process on one core and on the
host's cores.  ``--workload`` runs one workload alone.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GDSW-PCG solves/sec and M^-1 applies/sec at 1e-8 residual; p50/p99 solve latency"
# options.exact_order by name (values of the enum in include/gdsw.h)
ORDERS = {"natural": 0, "nd": 1, "auto": 2}

# HBM traffic of the dominant kernel measured with rocprofv3 FETCH_SIZE /
# WRITE_SIZE (calibrated by a device copy of known size; see
# profiles/hbm_traffic_*.md).  A figure only applies to the kernel source it
# was measured on: `src` is a hash of that kernel's text, checked below.
MEASURED_TRAFFIC = {
    ("k_ilu_jacobi", "poisson128^3_P8^3", "fp64"): {"bytes": 270263559, "src": "04585098cbd2f750"},
    ("k_ilu_jacobi", "poisson128^3_P8^3", "fp16"): {"bytes": 203127279, "src": "04585098cbd2f750"},
    ("k_band_apply", "poisson128^3_P8^3", "fp64"): {"bytes": 14214170851, "src": "af0e9d368f9e553e"},
    ("k_band_apply", "elasticity48^3", "fp32"): {"bytes": 1623322957, "src": "af0e9d368f9e553e"},
    ("k_nd_apply", "poisson128^3_P8^3", "fp64"): {"bytes": 5574150050, "src": "a6f6d04cf1931195"},
    ("k_nd_apply", "poisson128^3_P8^3", "fp16"): {"bytes": 1744098215, "src": "a6f6d04cf1931195"},
    # ILU(1) factors from 3 FastILU sweeps (the traffic does not depend on how the factors were computed)
    ("k_ilu_jacobi_phased", "poisson128^3_P8^3", "fp64"): {"bytes": 449873130, "src": "4e1cfa6c27b7f1c8"},
    # ILU(2) factors from 3 FastILU sweeps (the entry holds for ILU(2) only)
    ("k_ilu_jacobi_hold", "poisson128^3_P8^3", "fp64"): {"bytes": 1887125645, "src": "e771500e6d544bfb"},
}


def kernel_source_hash(kernel):
    """Hash of the source text a kernel is built from (its own text and the
    device functions it calls), to tie a counter measurement to a kernel."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2304_04876_amd", "csrc")
    segments = {
        "k_ilu_jacobi": [("kernels_apply.hpp", "template <int NT, int R, int KL, int KU, typename VT, bool MS>",
                          "// Same sweeps for any slot counts and subdomain sizes")],
        "k_band_apply": [("kernels_setup.hpp", "constexpr int BS_NB = 64;", "// Extension, eq. (2)."),
                         ("kernels_apply.hpp", "// Exact local solve A_i^{-1} r_i with the banded Cholesky factor",
                          "// Coarse restriction Phi^T r.")],
        "k_nd_apply": [("kernels_nd.hpp", "// Sum over aligned groups of G lanes", "}  // namespace gdsw")],
        "k_ilu_jacobi_phased": [("kernels_apply.hpp", "// The register-resident sweeps for factors with more slots",
                                 "// Exact local solve A_i^{-1} r_i with the banded Cholesky factor")],
        "k_ilu_jacobi_hold": [("kernels_apply.hpp", "// ILU(k) factors with more slots per row than the registers hold",
                               "// The register-resident sweeps for factors with more slots")],
    }
    if kernel not in segments:
        return None
    h = hashlib.sha256()
    for fname, start, end in segments[kernel]:
        text = open(os.path.join(csrc, fname)).read()
        a, b = text.find(start), text.find(end)
        if a < 0 or b < a:
            return None   # the kernel's text moved: no measurement applies to it
        h.update(text[a:b].encode())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)



GOLD = os.path.join(ROOT, "tests", "golden")


def single(kind="poisson", N=None, Pn=None, local="ilu0", prec="fp64", coarse=None, gmres="single_reduce",
           ilu_level=0, factor_sweeps=0, graphs=False, steps=10, warmup=2, kernel_reps=50, autotune=True,
           with_graph_apply=True, order="natural", element_sharing=False):
    """One workload on one handle: setup, autotune, `warmup` + `steps` timed
    solves, applies/s from a graph-replayed apply, the dominant kernel timed
    where it runs, and the error against FP64 oracle samples where the
    workload has them.  Returns a dict (the fields of the JSON line)."""
    import torch
    from paper_2304_04876_amd import binding as B
    from paper_2304_04876_amd import problems as P

    precs = {"fp64": B.FP64, "fp32": B.FP32, "bf16": B.BF16, "fp16": B.FP16}
    pbytes = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}[prec]
    loc = B.LOCAL_ILU0 if local == "ilu0" else B.LOCAL_EXACT
    elastic = kind == "elasticity"
    coarse_name = coarse or ("rgdsw" if elastic else "gdsw")
    if elastic:
        N, Pn = N or 48, Pn or 6
        log(f"[bench] building Q1 elasticity {N}^3 with {Pn}^3 boxes ({prec} {local} factors)")
        pr = P.elasticity_q1(N, Pn)
        Z = P.rigid_body_modes(pr)
        krylov = B.KRYLOV_GMRES_SR if gmres == "single_reduce" else B.KRYLOV_GMRES
    else:
        N, Pn = N or 128, Pn or 8
        log(f"[bench] building Poisson {N}^3 with {Pn}^3 boxes ({prec} {local} factors)")
        pr = P.poisson3d(N, Pn)
        Z = None
        krylov = B.KRYLOV_CG
    n = pr.n
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    sharing = P.element_sharing(pr) if element_sharing else None
    h = B.gdsw_analyze(pr.A, pr.part, pr.n_parts, pr.dpn, Z,
                       B.gdsw_default_options(local=loc, local_prec=precs[prec],
                                              basis_prec=B.FP64 if prec == "fp64" else B.FP32,
                                              ilu_level=ilu_level, ilu_factor_sweeps=factor_sweeps,
                                              coarse=B.COARSE_RGDSW if coarse_name == "rgdsw" else B.COARSE_GDSW,
                                              flags=B.FLAG_GRAPHS if graphs else 0,
                                              exact_order=ORDERS[order]),
                       sharing=sharing)
    t_an = time.perf_counter() - t0
    log(f"[bench] analysis {t_an:.2f}s; numerical setup on the GPU")
    B.gdsw_factor(h, stream)
    info = B.gdsw_get_info(h)
    log(f"[bench] setup {info['t_factor']:.3f}s  n0={info['n0']}  device bytes={info['device_bytes'] / 1e9:.2f} GB")
    if autotune:
        tune_ms = B.gdsw_autotune(h, reps=5, stream=stream)
        info = B.gdsw_get_info(h)
        log(f"[bench] autotune (ms per launch) {[round(t, 4) for t in tune_ms]} -> local variant "
            f"{info['local_variant']}, gemv variant {info['gemv_variant']}, "
            f"prolongation variant {info['prolong_variant']}")

    nrhs = warmup + steps
    if elastic:
        # the assembled body-force load, scaled per step so that every solve
        # starts from a different right-hand side
        rhs = torch.stack([torch.from_numpy(pr.b * (1.0 + 0.1 * s)) for s in range(nrhs)]).to(dev)
    else:
        rhs = torch.stack([torch.from_numpy(P.rhs_uniform(n, s)) for s in range(nrhs)]).to(dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    for k in range(warmup):
        B.gdsw_solve(h, rhs[k], x, krylov=krylov, restart=30, rtol=1e-8, maxit=2000, stream=stream)
    torch.cuda.synchronize()
    log(f"[bench] timing {steps} solves")
    iters, res_true = [], []
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        evs[k][0].record(stream)
        out = B.gdsw_solve(h, rhs[warmup + k], x, krylov=krylov, restart=30, rtol=1e-8, maxit=2000,
                           stream=stream)
        evs[k][1].record(stream)
        iters.append(out["iterations"])
        res_true.append(out["rel_res_true"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = [a.elapsed_time(b) for a, b in evs]
    assert max(res_true) <= 1.5e-8, res_true

    # ---- applies/s: hipGraph-replayed apply -------------------------------------
    r = rhs[0].clone()
    z_eager = torch.zeros_like(r)
    z = torch.zeros_like(r)
    B.gdsw_apply(h, r, z_eager, stream)
    torch.cuda.synchronize()
    apply_ms = None
    if with_graph_apply:
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            B.gdsw_apply(h, r, z, side)     # warm the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            B.gdsw_apply(h, r, z, torch.cuda.current_stream())
        torch.cuda.synchronize()
        reps = 200
        for _ in range(3):
            z.zero_()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(z, z_eager), "graph replay differs from the eager apply"
        times = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps // 5):
                graph.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / (reps // 5))
        apply_ms = float(np.median(times))
        del graph

    # ---- error against the FP64 oracle (sampled) ------------------------------------
    err = None
    xe = torch.zeros_like(r)
    if elastic and (N, Pn) == (48, 6) and not element_sharing:
        gold = np.load(os.path.join(GOLD, "elasticity_oracle.npz" if coarse_name == "gdsw"
                                    else f"elasticity_{coarse_name}_oracle.npz"))
        bl = torch.from_numpy(pr.b).to(dev)
        zl = torch.zeros_like(bl)
        B.gdsw_apply(h, bl, zl, stream)
        oe = B.gdsw_solve(h, bl, xe, krylov=krylov, restart=30, rtol=1e-8, maxit=2000, stream=stream)
        torch.cuda.synchronize()
        idx = torch.from_numpy(gold["idx"]).to(dev)
        err = {"apply_rel": float(np.abs(zl[idx].cpu().numpy() - gold["z"]).max() / float(gold["z_norm"])),
               "solution_rel": float(np.abs(xe[idx].cpu().numpy() - gold["x_gm"]).max() / float(gold["x_norm"])),
               "iterations": int(oe["iterations"]), "oracle_iterations": int(gold["gm_iters"]),
               "sample": "4096 seeded dofs; max-norm error relative to the oracle's max-norm; the oracle's "
                         "FP64 GMRES(30) solution to 1e-8 with the assembled load"}
    elif not elastic and (N, Pn) == (128, 8) and ilu_level == 0 and factor_sweeps == 0:
        gold = np.load(os.path.join(GOLD, "large_poisson_oracle.npz" if local == "ilu0"
                                    else "large_poisson_exact_oracle.npz"))
        b0 = torch.from_numpy(P.rhs_uniform(n, 0)).to(dev)
        z0 = torch.zeros_like(b0)
        B.gdsw_apply(h, b0, z0, stream)
        oe = B.gdsw_solve(h, b0, xe, krylov=krylov, rtol=1e-8, maxit=2000, stream=stream)
        torch.cuda.synchronize()
        idx = torch.from_numpy(gold["idx"]).to(dev)
        zkey = "z_ilu0" if local == "ilu0" else "z_exact"
        # the oracle's CG iterate after its own iteration count (its solution)
        xs = xe[idx].cpu().numpy()
        err = {"apply_rel": float(np.abs(z0[idx].cpu().numpy() - gold[zkey]).max() / float(gold["z_norm"])),
               "solution_rel": float(np.abs(xs - gold["x_fixed"]).max() / np.abs(gold["x_fixed"]).max()),
               "iterations": int(oe["iterations"]), "oracle_iterations": int(gold["cg_iters"][0]),
               "sample": "4096 seeded dofs, right-hand side 0; max-norm error relative to the oracle's "
                         "max-norm; the oracle's FP64 CG solution to 1e-8"}
    if err is not None:
        log(f"[bench] error vs oracle {err}")

    # ---- numeric re-setup: the numerical phase again on the same pattern
    # (here the same values), keeping maps, buffers and tuned launches
    A_sorted = pr.A.tocsr()
    A_sorted.sort_indices()
    B.gdsw_refactor(h, A_sorted.data, stream)
    torch.cuda.synchronize()
    t_refactor = B.gdsw_get_info(h)["t_refactor"]

    # ---- dominant kernel: the batched local solves, timed where they run ------------
    # HIP event pairs around the local-solve launch inside whole applies (the
    # coarse chain and the prolongation run between two launches, as in the
    # solves), on the stream they are launched on; for comparison also
    # back-to-back launches of the local solves alone, where part of the
    # factors can still be held in the 256 MB last-level cache from the launch
    # before
    B.gdsw_profile_local(h, True)
    for _ in range(kernel_reps):
        B.gdsw_apply(h, r, z, stream)
    k_durations = B.gdsw_profile_read(h)
    B.gdsw_profile_local(h, False)
    assert k_durations.size == kernel_reps, k_durations.size
    k_ms = float(np.mean(k_durations))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    B.gdsw_apply_part(h, r, None, 4, stream)
    e0.record(stream)
    for _ in range(kernel_reps):
        B.gdsw_apply_part(h, r, None, 4, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms_alone = e0.elapsed_time(e1) / kernel_reps
    nloc = info["sum_overlap_dofs"]
    # algorithmic bytes of one local-solve launch, from the library: ILU(0):
    # every stored off-diagonal factor entry once (value + 16-bit local
    # column) and the inverse pivot per local row; exact: the band twice
    # (forward, backward), or the supernodal panels' lower parts twice and
    # their gather lists and struct rows once; and per local row the
    # restriction index (4 B), the gathered r (8 B), the local result (8 B)
    alg_bytes = info["local_solve_bytes"]
    if local == "ilu0":
        if info["local_variant"] in (0, 1):
            # ILU(0): every entry in registers; ILU(1) (6 + 6 slots): L and
            # U entries in registers one after the other; ILU(2) and up: the
            # first slots of each row held, the others read on every sweep
            kname = {0: "k_ilu_jacobi", 1: "k_ilu_jacobi_phased"}.get(ilu_level, "k_ilu_jacobi_hold")
        else:
            kname = "k_ilu_jacobi_generic"
    elif info["nd_subdomains"] == pr.n_parts:
        kname = "k_nd_apply"
    elif info["nd_subdomains"] == 0:
        kname = "k_band_apply"
    else:
        kname = "k_band_apply+k_nd_apply"
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    # the whole apply (graph-replayed): local solves, coarse restriction
    # (Phi once + row index and r per row), A_0^{-1} GEMV, prolongation
    # (local results and their positions, dof maps, Phi again, z)
    s_phi = 8 if prec == "fp64" else 4
    apply_bytes = (alg_bytes + 2 * info["phi_entries"] * s_phi + n * 12 + 8 * info["n0"] ** 2
                   + nloc * 12 + n * 20)
    traffic = None
    meas = None
    if ((ilu_level == 0 and factor_sweeps == 0) or (kname == "k_ilu_jacobi_phased" and ilu_level == 1)
            or (kname == "k_ilu_jacobi_hold" and ilu_level == 2)):
        meas = MEASURED_TRAFFIC.get((kname, f"poisson{N}^3_P{Pn}^3" if not elastic else f"elasticity{N}^3", prec))
    if meas and kernel_source_hash(kname) == meas["src"]:
        traffic = int(meas["bytes"])
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": int(alg_bytes), "avg_launch_ms": round(k_ms, 5),
                "avg_launch_ms_back_to_back": round(k_ms_alone, 5)}
    local_name = local
    if local == "exact" and order != "natural":
        local_name = f"exact_{order}"
    if local == "ilu0" and (ilu_level or factor_sweeps):
        local_name = f"ilu{ilu_level}" + (f"_fast{factor_sweeps}" if factor_sweeps else "")
    out = {
        "value": round(steps / wall, 3),
        "ms_per_step": round(1e3 * wall / steps, 3),
        "steps": steps, "warmup": warmup,
        "dtype": "f64" if prec == "fp64" else f"f64+{prec}",
        "config": {"workload": (f"elasticity_q1_{N}^3_P{Pn}^3_{local}_{coarse_name}_gmres30"
                                f"{'_single_reduce' if gmres == 'single_reduce' else ''}" if elastic
                                else f"poisson{N}^3_P{Pn}^3_{local_name}_{coarse_name}_cg"), "n": n,
                   "n_parts": pr.n_parts, "n0": info["n0"], "overlap": 1, "local": local,
                   "jacobi_sweeps": 5, "ilu_level": ilu_level, "ilu_factor_sweeps": factor_sweeps,
                   "local_prec": prec, "rtol": 1e-8,
                   "exact_order": order if local == "exact" else None,
                   "interface": "element sharing sets" if element_sharing else "node graph",
                   "nd_subdomains": info["nd_subdomains"],
                   "tuned_local_variant": info["local_variant"], "tuned_gemv_variant": info["gemv_variant"],
                   "tuned_apply_streams": info["apply_streams"], "tuned_prolong_variant": info["prolong_variant"],
                   "graphs": bool(graphs)},
        "applies_per_sec": round(1e3 / apply_ms, 1) if apply_ms else None,
        "apply_ms": round(apply_ms, 4) if apply_ms else None,
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "latency_kind": "closed loop: one solve after another, each timed from its start on the stream",
        "iterations": int(np.median(iters)),
        "rel_res_true_max": float(max(res_true)),
        "setup_s": round(info["t_factor"], 3),
        "refactor_s": round(t_refactor, 3),
        "analysis_s": round(t_an, 3),
        "device_bytes": int(info["device_bytes"]),
        "roofline": roofline,
        "apply_roofline": ({"bound": "hbm", "alg_bytes_per_apply": int(apply_bytes),
                            "achieved": round(apply_bytes / (apply_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(apply_bytes / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
                           if apply_ms else None),
    }
    if err is not None:
        out["error_vs_oracle"] = err
    B.gdsw_destroy(h)
    del rhs, x, xe, r, z, z_eager
    torch.cuda.synchronize()
    return out


def cpu_baseline(kind="poisson", N=128, Pn=8, local="ilu0", coarse="gdsw", gmres="single_reduce",
                 ilu_level=0, factor_sweeps=0, seed=2):
    """The FP64 oracle on the host, in a child process (no GPU context):
    one full solve with the serial subdomain loop (1 core) and one with the
    loop over worker processes on the host's cores (at most 16)."""
    import subprocess
    cmd = [sys.executable, "-m", "oracle.cpu_baseline", "--workload", kind, "--N", str(N), "--P", str(Pn),
           "--local", local, "--coarse", coarse, "--gmres", gmres, "--ilu-level", str(ilu_level),
           "--factor-sweeps", str(factor_sweeps), "--seed", str(seed)]
    log("[bench] CPU oracle in a child process: " + " ".join(cmd[1:]))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    if res.returncode != 0:
        log(res.stderr[-2000:])
        raise RuntimeError(f"CPU baseline failed ({res.returncode})")
    c = json.loads(res.stdout.strip().splitlines()[-1])
    return {"value": c["parallel_solves_per_s"], "unit": "solves/s", "cores": c["workers"], "kind": "oracle",
            "sample": (f"one full FP64 oracle solve of the same workload (right-hand side {seed}, "
                       f"{c['iterations']} iterations, {c['parallel_s']} s) with the subdomain loop over "
                       f"{c['workers']} worker processes, preconditioner set up beforehand (untimed, "
                       f"{c['setup_s']} s); BLAS one thread per process"),
            "one_core": {"value": c["serial_solves_per_s"], "seconds": c["serial_s"]},
            "cores_available": c["cores_available"], "nproc": c["nproc"], "cpu_model": c["cpu_model"],
            "iterations": c["iterations"]}


def sub(d, keys=("value", "ms_per_step", "dtype", "applies_per_sec", "p50_ms", "p99_ms", "iterations",
                 "rel_res_true_max", "setup_s", "device_bytes", "error_vs_oracle")):
    out = {k: d[k] for k in keys if k in d and d[k] is not None}
    out["workload"] = d["config"]["workload"]
    out["unit"] = "solves/s"
    out["roofline"] = {k: d["roofline"][k] for k in ("kernel", "achieved", "frac", "avg_launch_ms", "traffic",
                                                     "alg_bytes_per_launch")}
    if d.get("apply_roofline"):
        out["apply_roofline_frac"] = d["apply_roofline"]["frac"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--local", choices=["ilu0", "exact"], default=None,
                    help="local solver (default: ilu0 for Poisson, exact for elasticity)")
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16", "fp16"], default="fp64")
    ap.add_argument("--exact-order", choices=["natural", "nd", "auto"], default="natural",
                    help="exact local solves: band Cholesky in the natural order, the supernodal Cholesky "
                         "after nested dissection, or per subdomain the one with fewer factor values")
    ap.add_argument("--workload", choices=["all", "poisson", "elasticity", "batch", "serve"], default="all",
                    help="all (default): the headline line with the other workloads as sub-records")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-exact-order", choices=["natural", "nd", "auto"], default="nd",
                    help="batch workload: ordering of the exact local factors (the supernodal factor after "
                         "nested dissection by default, the experiments' choice for exact solvers)")
    ap.add_argument("--batch-seq-stride", type=int, default=1,
                    help="batch workload: time the sequential FP64 reference on every k-th problem")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--graphs", action="store_true", help="queue CG iterations as captured HIP graphs")
    ap.add_argument("--gmres", choices=["single_reduce", "classical"], default="single_reduce",
                    help="GMRES variant of the elasticity workload: one reduction per iteration (the "
                         "paper's experiments) or classical Gram-Schmidt applied twice")
    ap.add_argument("--coarse", choices=["gdsw", "rgdsw"], default=None,
                    help="coarse space: GDSW, or the reduced GDSW space of the paper's experiments "
                         "(default: rgdsw for the elasticity workload, gdsw for Poisson)")
    ap.add_argument("--element-sharing", action="store_true",
                    help="elasticity: the interface from the element decomposition's sharing sets (the "
                         "geometric GDSW / rGDSW space) instead of the node graph")
    ap.add_argument("--ilu-level", type=int, default=0)
    ap.add_argument("--factor-sweeps", type=int, default=0)
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--P", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU sharding "
                          "of the preconditioner is a design note only (--gpus must be 1)"}))
        sys.exit(2)

    if args.workload == "batch":
        print(json.dumps(bench_batch(args, sequential_stride=args.batch_seq_stride)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    kind = "elasticity" if args.workload == "elasticity" else "poisson"
    if args.local is None:
        args.local = "exact" if kind == "elasticity" else "ilu0"
    d = single(kind, args.N, args.P, args.local, args.prec, args.coarse, args.gmres, args.ilu_level,
               args.factor_sweeps, args.graphs, args.steps, args.warmup, args.kernel_reps,
               order=args.exact_order, element_sharing=args.element_sharing)
    line = {
        "metric": METRIC,
        "value": d["value"], "unit": "solves/s", "n_gpus": 1, "steps": d["steps"], "warmup": d["warmup"],
        "ms_per_step": d["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": d["dtype"], "data": "synthetic", "config": d["config"],
    }
    for k, v in d.items():
        if k not in line and k not in ("steps", "warmup"):
            line[k] = v
    if args.workload == "all":
        # the other workloads, at reduced step counts
        fp16 = single("poisson", args.N, args.P, "ilu0", "fp16", steps=max(3, args.steps // 2), warmup=1,
                      kernel_reps=20)
        line["mixed_precision_fp16"] = sub(fp16)
        line["mixed_precision_fp16"]["vs_fp64_solves_per_s"] = round(fp16["value"] / d["value"], 3)
        # exact local solves: the supernodal factor after nested dissection
        # (the faster form on these 16^3 boxes) and the band beside it
        line["iluk_fastilu"] = sub(single("poisson", args.N, args.P, "ilu0", "fp64", None, "single_reduce", 1, 3,
                                          steps=3, warmup=1, kernel_reps=10))
        # ILU(2): 11 + 11 factor entries per row, more than registers and LDS
        # hold, so the streaming sweeps read the factors on every sweep
        line["iluk2_fastilu"] = sub(single("poisson", args.N, args.P, "ilu0", "fp64", None, "single_reduce", 2, 3,
                                           steps=2, warmup=1, kernel_reps=10))
        line["exact_local"] = sub(single("poisson", args.N, args.P, "exact", "fp64", steps=3, warmup=1,
                                         kernel_reps=10, order="nd"))
        line["exact_local_band"] = sub(single("poisson", args.N, args.P, "exact", "fp64", steps=3, warmup=1,
                                              kernel_reps=10, order="natural"))
        # mixed precision on the exact form: FP16 supernodal factors (FP32
        # accumulation), FP64 CG
        ex16 = single("poisson", args.N, args.P, "exact", "fp16", steps=3, warmup=1, kernel_reps=10, order="nd")
        line["exact_local_fp16"] = sub(ex16)
        line["exact_local_fp16"]["vs_fp64_solves_per_s"] = round(ex16["value"] / line["exact_local"]["value"], 3)
        line["elasticity"] = sub(single("elasticity", None, None, "exact", "fp32", None, "single_reduce",
                                        steps=3, warmup=1, kernel_reps=10))
        bargs = argparse.Namespace(**vars(args))
        bargs.steps = 1
        line["batch"] = bench_batch(bargs, sequential_stride=8)
        sargs = argparse.Namespace(**vars(args))
        sargs.serve_requests, sargs.serve_warmup = 300, 40
        line["serving"] = bench_serve(sargs, quick=True)
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(kind, args.N or (48 if kind == "elasticity" else 128),
                           args.P or (6 if kind == "elasticity" else 8), args.local,
                           args.coarse or ("rgdsw" if kind == "elasticity" else "gdsw"), args.gmres,
                           args.ilu_level, args.factor_sweeps, seed=args.warmup)
        if abs(cpu["iterations"] - d["iterations"]) > 1 and args.prec == "fp64":
            log(f"[bench] WARNING: GPU iterations {d['iterations']} vs oracle {cpu['iterations']}")
        line["cpu_baseline"] = cpu
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


def bench_batch(args, sequential_stride=1):
    """256 independent diffusion problems (N in [16,48], P in [2,4], kappa =
    exp(N(0,1)) per cell), exact local factors stored FP32, FP64 CG: all
    problems packed in one handle and solved together, against the same
    problems solved one after another with one FP64 handle each (every
    `sequential_stride`-th problem, rate scaled to the whole batch); the
    FP32 solutions of eight problems are compared with FP64 oracle samples."""
    import torch
    from paper_2304_04876_amd import binding as B
    from paper_2304_04876_amd import problems as P

    log(f"[batch] generating {args.batch_count} diffusion problems")
    specs = P.batch_diffusion_specs(args.batch_count)
    probs = [P.batch_diffusion_problem(sp) for sp in specs]
    t0 = time.perf_counter()
    hb = B.gdsw_analyze_batch([(p.A, p.part, p.n_parts) for p in probs],
                              options=B.gdsw_default_options(local=B.LOCAL_EXACT, local_prec=B.FP32,
                                                             basis_prec=B.FP32,
                                                             flags=B.FLAG_GRAPHS if args.graphs else 0,
                                                             exact_order=ORDERS[args.batch_exact_order]))
    t_an = time.perf_counter() - t0
    B.gdsw_factor(hb)
    tune = B.gdsw_autotune(hb, reps=3)
    info = B.gdsw_get_info(hb)
    log(f"[batch] n={info['n']} subdomains={info['n_parts']} analysis {t_an:.1f}s setup {info['t_factor']:.2f}s "
        f"device {info['device_bytes'] / 1e9:.1f} GB; autotune {[round(t, 3) for t in tune[:6]]}")
    offs = B.gdsw_problem_offsets(hb)
    b = torch.from_numpy(np.concatenate([p.b for p in probs])).cuda()
    x = torch.zeros_like(b)
    B.gdsw_solve_batch(hb, b, x, rtol=1e-8, maxit=2000)      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(1, args.steps)
    for _ in range(reps):
        infos = B.gdsw_solve_batch(hb, b, x, rtol=1e-8, maxit=2000)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    res = max(i["rel_res_true"] for i in infos)
    its = [i["iterations"] for i in infos]
    # error of the FP32-factor solutions against FP64 oracle samples
    errs = {}
    if args.batch_count == 256:
        gold = np.load(os.path.join(GOLD, "batch_serve_oracle.npz"))
        xh = x.cpu().numpy()
        for j, k in enumerate(gold["batch_k"]):
            k = int(k)
            xs = xh[offs[k]:offs[k + 1]][gold["batch_idx"][j]]
            errs[str(k)] = {"N": int(specs[k]["N"]), "P": int(specs[k]["P"]),
                            "rel_err": float(np.abs(xs - gold["batch_x"][j]).max() / float(gold["batch_x_norm2"][j])),
                            "iterations": int(its[k]), "oracle_iterations": int(gold["batch_iters"][j])}
    B.gdsw_destroy(hb)
    # the same problems one at a time, FP64 local factors, one handle each
    log("[batch] sequential FP64 reference")
    seq, seq_res, nseq = 0.0, 0.0, 0
    for k in range(0, len(probs), sequential_stride):
        p = probs[k]
        g = B.Gdsw(p.A, p.part, p.n_parts, 1, local=B.LOCAL_EXACT, exact_order=ORDERS[args.batch_exact_order])
        bk = b[int(offs[k]):int(offs[k + 1])].clone()
        xk = torch.zeros_like(bk)
        g.solve(bk, xk, rtol=1e-8, maxit=2000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = g.solve(bk, xk, rtol=1e-8, maxit=2000)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t0
        seq_res = max(seq_res, out["rel_res_true"])
        nseq += 1
        g.close()
    seq_rate = nseq / seq
    return {
        "metric": METRIC,
        "value": round(len(probs) / wall, 2), "unit": "solves/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": round(1e3 * wall, 2), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+fp32", "data": "synthetic",
        "config": {"workload": f"batch{len(probs)}_diffusion_N16-48_P2-4_exact"
                               f"{'' if args.batch_exact_order == 'natural' else '_' + args.batch_exact_order}"
                               "_fp32_gdsw_cg",
                   "n": int(info["n"]), "n_parts": int(info["n_parts"]), "rtol": 1e-8,
                   "graphs": bool(args.graphs), "exact_order": args.batch_exact_order,
                   "nd_subdomains": int(info["nd_subdomains"]),
                   "local_classes": int(info["local_classes"])},
        "iterations_min_median_max": [int(min(its)), int(np.median(its)), int(max(its))],
        "rel_res_true_max": res,
        "sequential_fp64_solves_per_s": round(seq_rate, 2),
        "sequential_fp64_problems_timed": nseq,
        "sequential_fp64_rel_res_true_max": seq_res,
        "vs_sequential_fp64": round(len(probs) / wall / seq_rate, 2),
        "error_vs_oracle": {"per_problem": errs,
                            "sample": "512 seeded dofs per problem; max error relative to the oracle solution's "
                                      "2-norm; the oracle's FP64 CG solution to 1e-8 with exact local solves"},
        "setup_s": round(info["t_factor"], 3), "analysis_s": round(t_an, 2),
        "device_bytes": int(info["device_bytes"]),
    }


def bench_serve(args, quick=False):
    """Serving stream over 8 resident Poisson operators (N = 32..96,
    P = round(N/16)), ILU(0) local factors in FP16 with FP32 arithmetic,
    FP64 CG to 1e-8; Poisson arrivals at 0.5 and 0.8 of the measured
    saturation rate (latency = completion - arrival); the same requests
    solved one at a time with FP64 handles (no batching) for comparison; a
    run whose slot count comes from a small HBM budget; three requests
    compared with FP64 oracle samples."""
    import torch
    from paper_2304_04876_amd import binding as B
    from paper_2304_04876_amd import problems as P
    from paper_2304_04876_amd import serve as SV

    ops = [P.serve_operator(N) for N in P.SERVE_SIZES]
    log("[serve] operators " + ", ".join(f"{p.name} n={p.n}" for p in ops))
    srv = SV.Server(ops, slots_per_op=4, local=B.LOCAL_ILU0, local_prec=B.FP16, basis_prec=B.FP32,
                    graphs=args.graphs)
    gold = np.load(os.path.join(GOLD, "batch_serve_oracle.npz"))
    gold_ops = {int(N): j for j, N in enumerate(gold["serve_N"])}

    def make(nreq, rate, seed):
        t, opi = SV.poisson_arrivals(nreq, rate, len(ops), seed)
        return [SV.Request(rid=i, op=int(opi[i]), arrival=float(t[i]),
                           b=P.rhs_uniform(ops[int(opi[i])].n, i)) for i in range(nreq)]

    # saturation: everything arrives at once
    sat_n = 8 * 4 * 3
    reqs, _ = srv.run(make(sat_n, 1e9, 1))
    mu = SV.summarize(reqs, srv).solves_per_s
    log(f"[serve] saturation {mu:.1f} solves/s")
    out = {}
    err = {}
    for frac in (0.5, 0.8):
        nreq = args.serve_requests + args.serve_warmup
        reqs = make(nreq, frac * mu, 2)
        keep = set()
        if frac == 0.5:
            # the oracle's three requests replace three measured ones
            # (operators N = 32, 59, 96; right-hand sides rhs_uniform(n, rid))
            for j, N in enumerate(gold["serve_N"]):
                k = args.serve_warmup + 10 + 25 * j
                q = reqs[k]
                q.op = P.SERVE_SIZES.index(int(N))
                q.rid = int(gold["serve_rid"][j])
                q.b = P.rhs_uniform(ops[q.op].n, q.rid)
                keep.add(q.rid)
        reqs, sols = srv.run(reqs, keep_solutions=keep)
        st = SV.summarize(reqs, srv, skip=args.serve_warmup)
        out[frac] = st
        for q in reqs:
            if q.rid in sols:
                j = gold_ops[P.SERVE_SIZES[q.op]]
                xs = sols[q.rid].cpu().numpy()[gold["serve_idx"][j]]
                err[f"N={P.SERVE_SIZES[q.op]}"] = {
                    "rel_err": float(np.abs(xs - gold["serve_x"][j]).max() / float(gold["serve_x_norm2"][j])),
                    "iterations": int(q.iterations), "oracle_iterations": int(gold["serve_iters"][j])}
        log(f"[serve] load {frac}: {st.solves_per_s:.1f} solves/s p50 {st.p50_ms:.1f} ms p99 {st.p99_ms:.1f} ms")
    slots_bytes = srv.device_bytes
    srv.close()
    # a small HBM budget: admission by the budget gives one slot per operator
    probe = SV.Server(ops, slots_per_op=1, local=B.LOCAL_ILU0, local_prec=B.FP16, basis_prec=B.FP32)
    one = probe.device_bytes
    probe.close()
    small = SV.Server(ops, hbm_budget_bytes=int(1.5 * one), local=B.LOCAL_ILU0, local_prec=B.FP16,
                      basis_prec=B.FP32, graphs=args.graphs)
    reqs, _ = small.run(make(200 if quick else 400, 0.5 * mu, 3))
    st_small = SV.summarize(reqs, small, skip=25 if quick else 50)
    small_slots, small_bytes = small.slots_per_op, small.device_bytes
    small.close()
    # plain FP64 GPU path: the same kind of requests one at a time
    log("[serve] sequential FP64 reference")
    handles = [B.Gdsw(p.A, p.part, p.n_parts, 1, local=B.LOCAL_ILU0) for p in ops]
    reqs = make(80 if quick else 160, 1e9, 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    resmax = 0.0
    for r in reqs:
        bd = torch.from_numpy(r.b).cuda()
        xd = torch.zeros_like(bd)
        o = handles[r.op].solve(bd, xd, rtol=1e-8)
        resmax = max(resmax, o["rel_res_true"])
    torch.cuda.synchronize()
    seq_rate = len(reqs) / (time.perf_counter() - t0)
    for g in handles:
        g.close()
    s5 = out[0.5]
    return {
        "metric": METRIC,
        "value": round(s5.solves_per_s, 2), "unit": "solves/s", "n_gpus": 1, "steps": args.serve_requests,
        "warmup": args.serve_warmup, "ms_per_step": round(1e3 / s5.solves_per_s, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+fp16", "data": "synthetic",
        "config": {"workload": "serve8_poisson32-96_ilu0_fp16_gdsw_cg", "slots_per_op": 4, "rtol": 1e-8,
                   "graphs": bool(args.graphs), "step_iters": srv.step_iters},
        "latency_kind": "completion - arrival (Poisson arrivals)",
        "saturation_solves_per_s": round(mu, 2),
        "load": {str(f): {"solves_per_s": round(v.solves_per_s, 2), "p50_ms": round(v.p50_ms, 2),
                          "p99_ms": round(v.p99_ms, 2), "mean_iters": round(v.mean_iters, 1),
                          "max_rel_res_true": v.max_rel_res_true} for f, v in out.items()},
        "small_budget": {"hbm_budget_bytes": int(1.5 * one), "slots_per_op": small_slots,
                         "device_bytes": int(small_bytes), "solves_per_s": round(st_small.solves_per_s, 2),
                         "p50_ms": round(st_small.p50_ms, 2), "p99_ms": round(st_small.p99_ms, 2)},
        "device_bytes_4_slots": int(slots_bytes),
        "sequential_fp64_solves_per_s": round(seq_rate, 2),
        "sequential_fp64_rel_res_true_max": resmax,
        "vs_sequential_fp64": round(s5.solves_per_s / seq_rate, 2),
        "saturation_vs_sequential_fp64": round(mu / seq_rate, 2),
        "error_vs_oracle": {"per_request": err,
                            "sample": "512 seeded dofs; max error relative to the oracle solution's 2-norm; "
                                      "the oracle's FP64 CG solution to 1e-8 (FP64 ILU(0) factors)"},
    }


if __name__ == "__main__":
    main()

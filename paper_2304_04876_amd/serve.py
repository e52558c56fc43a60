"""Serving loop: factored GDSW preconditioners stay resident on the GPU and
incoming right-hand sides are solved with continuous batching.

All operators sit in one handle of the library, factored once; the handle
holds S right-hand-side *slots* of every operator (its `slots` option): per
slot only the Krylov vectors and the apply's intermediate results, while
the local factors, the coarse basis, A_0^{-1} and the matrix are shared by
all slots of an operator (the register-resident local solves read each
factor entry once for all slots of a subdomain).  A request names an
operator and a right-hand side; it waits in that operator's queue until one
of its slots is free, is then loaded into the slot and started, and from
there on advances together with every other running slot: each step runs
``step_iters`` CG iterations of all running slots in shared kernel
launches.  A slot that converges returns its result at the next step
boundary and takes the next queued request at once.  S comes from an HBM
budget: the operators' resident bytes plus S slot workspaces (the library
reports both) must fit it.  Each slot's arithmetic is independent of what
the other slots hold, so a result is bit-identical alone and in the mix.

This module is driver code over the C ABI (``binding``): all numerical work
runs in the library's kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as B


@dataclass
class Request:
    rid: int
    op: int
    arrival: float            # seconds from the start of the run
    b: np.ndarray | None = None
    start: float = -1.0
    finish: float = -1.0
    iterations: int = 0
    rel_res_true: float = float("nan")
    status: int = -1


@dataclass
class ServeStats:
    completed: int
    wall: float
    solves_per_s: float
    p50_ms: float
    p99_ms: float
    mean_iters: float
    max_rel_res_true: float
    slots_per_op: int
    device_bytes: int
    latencies_ms: list = field(default_factory=list)


class Server:
    def __init__(self, operators, slots_per_op=None, hbm_budget_bytes=0, local=B.LOCAL_ILU0,
                 local_prec=B.FP16, basis_prec=B.FP32, rtol=1e-8, maxit=1000, step_iters=4,
                 stream=None, graphs=False, autotune=True):
        import torch
        self.torch = torch
        self.ops = operators
        self.rtol = rtol
        self.maxit = maxit
        self.step_iters = step_iters
        self.opts = dict(local=local, local_prec=local_prec, basis_prec=basis_prec,
                         flags=B.FLAG_GRAPHS if graphs else 0)
        self.stream = stream
        self.hbm_budget_bytes = int(hbm_budget_bytes)
        if slots_per_op is None:
            slots_per_op = self._slots_for_budget(hbm_budget_bytes)
        if slots_per_op < 1:
            raise B.GdswError(5, "HBM budget too small for one slot per operator")
        self.slots_per_op = slots_per_op
        nops = len(operators)
        self.h = B.gdsw_analyze_batch([(op.A, op.part, op.n_parts) for op in operators],
                                      options=B.gdsw_default_options(slots=slots_per_op, **self.opts))
        B.gdsw_factor(self.h, stream)
        if autotune:   # launch configurations timed on this handle, the same for every slot
            B.gdsw_autotune(self.h, reps=3, stream=stream)
        # Krylov problem v = k * nops + p: operator p in slot k
        self.offs = B.gdsw_problem_offsets(self.h)
        self.slot_op = [v % nops for v in range(slots_per_op * nops)]
        n = int(self.offs[-1])
        self.b = torch.zeros(n, dtype=torch.float64, device="cuda")
        self.x = torch.zeros_like(self.b)
        B.gdsw_slots_begin(self.h, self.b, self.x, rtol, maxit, stream)
        info = B.gdsw_get_info(self.h)
        # device bytes: the handle (operators once + per-slot workspaces)
        # and the right-hand sides and solutions of every slot
        self.device_bytes = info["device_bytes"] + 2 * 8 * n
        self.operator_bytes = info["device_bytes"] - slots_per_op * info["slot_bytes"]
        self.slot_workspace_bytes = info["slot_bytes"] + 2 * 8 * n // slots_per_op

    def _slots_for_budget(self, budget):
        """Slots per operator that fit `budget` device bytes (0: four): the
        operators' resident bytes and one slot's workspace are read from a
        one-slot probe handle."""
        if not budget:
            return 4
        probe = B.gdsw_analyze_batch([(op.A, op.part, op.n_parts) for op in self.ops],
                                     options=B.gdsw_default_options(slots=1, **self.opts))
        try:
            B.gdsw_factor(probe, self.stream)
            info = B.gdsw_get_info(probe)
        finally:
            B.gdsw_destroy(probe)
        n = sum(op.n for op in self.ops)
        resident = info["device_bytes"] - info["slot_bytes"]
        per_slot = info["slot_bytes"] + 2 * 8 * n
        return int((budget - resident) // per_slot)

    def close(self):
        if getattr(self, "h", None):
            B.gdsw_destroy(self.h)
            self.h = None

    def run(self, requests, keep_solutions=False):
        """Serves `requests` (sorted by arrival, seconds from now); returns
        the requests with their times and results filled in, and the
        solutions (device copies) of every request (keep_solutions=True) or
        of the request ids in the collection keep_solutions."""
        torch = self.torch
        nslot = len(self.slot_op)
        free = {k: [s for s in range(nslot) if self.slot_op[s] == k] for k in range(len(self.ops))}
        queues = {k: [] for k in range(len(self.ops))}
        running = {}
        pending = list(requests)
        pending.reverse()
        solutions = {}
        t0 = time.perf_counter()
        done = 0
        total = len(requests)
        while done < total:
            now = time.perf_counter() - t0
            while pending and pending[-1].arrival <= now:
                r = pending.pop()
                queues[r.op].append(r)
            # admission: free slots take queued requests of their operator
            for k in queues:
                while queues[k] and free[k]:
                    r = queues[k].pop(0)
                    s = free[k].pop()
                    lo, hi = int(self.offs[s]), int(self.offs[s + 1])
                    self.b[lo:hi].copy_(torch.from_numpy(r.b), non_blocking=False)
                    B.gdsw_slot_start(self.h, s, self.stream)
                    r.start = time.perf_counter() - t0
                    running[s] = r
            if not running:
                if pending:
                    wait = pending[-1].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            state = B.gdsw_slots_step(self.h, self.step_iters, self.stream)
            fin_t = time.perf_counter() - t0
            for s in list(running):
                if state[s] in (1, 2):
                    r = running.pop(s)
                    info = B.gdsw_slot_finish(self.h, s, self.stream)
                    r.finish = fin_t
                    r.iterations = info["iterations"]
                    r.rel_res_true = info["rel_res_true"]
                    r.status = info["status"]
                    if keep_solutions is True or (keep_solutions and r.rid in keep_solutions):
                        lo, hi = int(self.offs[s]), int(self.offs[s + 1])
                        solutions[r.rid] = self.x[lo:hi].clone()
                    free[self.slot_op[s]].append(s)
                    done += 1
        return requests, solutions


def poisson_arrivals(n_requests, rate, n_ops, seed=0):
    """Arrival times of a Poisson process of the given rate (requests/s)
    and uniformly drawn operators."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    ops = rng.integers(0, n_ops, n_requests)
    return t, ops


def summarize(reqs, server, skip=0) -> ServeStats:
    meas = [r for r in reqs[skip:] if r.finish >= 0]
    lat = np.array([1e3 * (r.finish - r.arrival) for r in meas])
    span = max(r.finish for r in meas) - min(r.arrival for r in meas)
    return ServeStats(completed=len(meas), wall=span, solves_per_s=len(meas) / span,
                      p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                      mean_iters=float(np.mean([r.iterations for r in meas])),
                      max_rel_res_true=float(max(r.rel_res_true for r in meas)),
                      slots_per_op=server.slots_per_op, device_bytes=int(server.device_bytes),
                      latencies_ms=lat.tolist())

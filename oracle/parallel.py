"""The oracle's apply with its subdomain loop spread over worker processes
(TEST INFRASTRUCTURE ONLY: used to time the CPU baseline on all host cores).

The one-level sum of eq. (1) is a loop over independent subdomains.  Here the
local solves z_i = A_i^{-1} R_i r of disjoint groups of subdomains run in
forked worker processes, each calling the oracle's own ``local_solve``; the
results land in a shared buffer, and the parent adds them into z in
ascending subdomain order and then adds the coarse term (computed while the
workers run) exactly as ``GDSW.apply`` does.  The arithmetic and its order are the serial oracle's,
so the result is bit-identical to ``GDSW.apply`` (tested).

Processes rather than threads: the ILU(0)-Jacobi local solves are many small
numpy operations that hold the interpreter lock.  Workers are forked after
the oracle is set up, so they share its factors copy-on-write.  Fork only
from a process that has not initialised a GPU.
"""
from __future__ import annotations

import multiprocessing as mp

import numpy as np
import scipy.linalg as sla


def _worker(M, ids, offs, r_buf, z_buf, n, tot, conn):
    r = np.frombuffer(r_buf, dtype=np.float64, count=n)
    zl = np.frombuffer(z_buf, dtype=np.float64, count=tot)
    while True:
        msg = conn.recv()
        if msg is None:
            break
        for i in ids:
            Ri = M.R[i]
            zl[offs[i]:offs[i] + Ri.size] = M.local_solve(i, r[Ri])
        conn.send(1)
    conn.close()


class ForkedApply:
    """z = M^{-1} r for an oracle GDSW object M with ``workers`` processes.
    Subdomains are dealt to workers in contiguous groups of about equal
    total size.  Use as a context manager (or call close())."""

    def __init__(self, M, workers: int):
        self.M = M
        ctx = mp.get_context("fork")
        sizes = np.array([Ri.size for Ri in M.R], dtype=np.int64)
        self.offs = np.concatenate([[0], np.cumsum(sizes)])
        tot = int(self.offs[-1])
        self._r = ctx.RawArray("d", max(M.n, 1))
        self._z = ctx.RawArray("d", max(tot, 1))
        self.r = np.frombuffer(self._r, dtype=np.float64, count=M.n)
        self.zl = np.frombuffer(self._z, dtype=np.float64, count=tot)
        workers = max(1, min(int(workers), len(M.R)))
        # contiguous groups of about tot / workers rows
        bounds = np.searchsorted(self.offs[1:], np.arange(1, workers) * tot / workers, side="left") + 1
        groups = np.split(np.arange(len(M.R)), bounds)
        self.conns, self.procs = [], []
        for ids in groups:
            if ids.size == 0:
                continue
            a, b = ctx.Pipe()
            p = ctx.Process(target=_worker, args=(M, ids.tolist(), self.offs, self._r, self._z, M.n, tot, b),
                            daemon=True)
            p.start()
            b.close()
            self.conns.append(a)
            self.procs.append(p)
        self.workers = len(self.procs)

    def apply(self, r: np.ndarray) -> np.ndarray:
        M = self.M
        self.r[:] = np.asarray(r, dtype=np.float64)
        for c in self.conns:
            c.send(1)
        # the coarse term meanwhile (an independent vector; added last, as
        # in the serial apply)
        zc = None
        if M.cs is not None:
            r0 = M.cs.phi.T @ self.r
            z0 = sla.cho_solve(M.A0_chol, r0)
            zc = M.cs.phi @ z0
        for c in self.conns:
            c.recv()
        z = np.zeros(M.n)
        for i, Ri in enumerate(M.R):
            if Ri.size:
                z[Ri] += self.zl[self.offs[i]:self.offs[i] + Ri.size]
        if zc is not None:
            z += zc
        return z

    def close(self):
        for c in self.conns:
            try:
                c.send(None)
                c.close()
            except (BrokenPipeError, OSError):
                pass
        for p in self.procs:
            p.join(timeout=10)
        self.conns, self.procs = [], []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

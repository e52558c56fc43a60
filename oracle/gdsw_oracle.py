"""Plain FP64 CPU oracle of the GDSW two-level overlapping additive Schwarz
preconditioner and the Krylov solvers it is used in.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct
reference the GPU library is checked against.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the GPU
library never calls it, and the two share no code (the oracle only reads the
seeded problem generators, which hold none of the method's arithmetic).

What it computes (paper: Sec. III, eqs. (1) and (2); Sec. V-B; Sec. VII):

    M^{-1} r = sum_i R_i^T A_i^{-1} R_i r + Phi A_0^{-1} Phi^T r,   A_0 = Phi^T A Phi,
    Phi = [ -A_II^{-1} A_IG ; I ] Phi_G.

Steps, in the order of the paper's construction:

  O1  node graph of the matrix pattern
  O2  overlapping subdomains: the nonoverlapping node partition grown by
      ``overlap`` layers of graph neighbours (Sec. III, first paragraph;
      the experiments use an algebraic overlap of one, Sec. VII)
  O3  local matrices A_i = R_i A R_i^T (eq. (1))
  O4  interface Gamma / interior I of the nonoverlapping partition (Sec. III)
  O5  interface components Gamma_1..Gamma_nc (Sec. III, item 1)
  O6  partition of unity D = I on disjoint components (Sec. III, item 2)
  O7  null space Z (Sec. III, item 3), supplied by the caller
  O8  Phi_Gamma_c spans D R_Gamma_c (R_Gamma Z) (Sec. III, item 4); O8r the
      reduced variant with coarse functions for the vertices only (Sec. III,
      variants of GDSW)
  O9  energy-minimising extension, eq. (2), with A_II block diagonal
  O10 coarse matrix A_0 = Phi^T A Phi (the paper prints Phi A Phi^T; only
      Phi^T A Phi has the right shape for eq. (1))
  O11 local factors: exact (sparse LU, a library primitive) or level-based
      ILU(k) (Sec. V-B, "Incomplete Local Solver"; k = 0 by default, Sec.
      VII-C varies it), computed exactly (row by row) or by the iterative
      FastILU variant (Jacobi sweeps on the factor entries, Sec. V-B)
  O12 coarse factor: dense Cholesky
  O13 apply, eq. (1); with ILU(0) the two triangular solves are done by
      Jacobi sweeps from a zero start (Sec. V-B: five iterations by default)
  O14 preconditioned CG and right-preconditioned GMRES(m); O14b the
      single-reduce GMRES(m) of the experiments (Sec. VII)

Readings where the paper is silent or inconsistent are stated at each step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def build_c(force: bool = False) -> str:
    """Compile the oracle's plain C helpers (incomplete LU) with gcc."""
    so = os.path.join(_HERE, "liboracle.so")
    src = os.path.join(_HERE, "ilu.c")
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        tmp = so + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, so)
    return so


def _lib():
    global _LIB
    if _LIB is None:
        _LIB = ctypes.CDLL(build_c())
        _LIB.oracle_ilu0.restype = ctypes.c_int
        _LIB.oracle_ilu0.argtypes = [ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
        _LIB.oracle_iluk_pattern.restype = ctypes.c_int64
        _LIB.oracle_iluk_pattern.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    return _LIB


# ---------------------------------------------------------------------------
# O1-O5: graph, overlap, interface, components
# ---------------------------------------------------------------------------

def node_graph(A: sp.csr_matrix, dpn: int) -> sp.csr_matrix:
    """O1: nodes u ~ v (u != v) iff a stored entry of A couples a dof of u with
    a dof of v; the pattern is taken as stored and symmetrised."""
    A = sp.csr_matrix(A)
    coo = A.tocoo()
    u = coo.row // dpn
    v = coo.col // dpn
    keep = u != v
    nn = A.shape[0] // dpn
    G = sp.coo_matrix((np.ones(int(keep.sum()), dtype=np.int8), (u[keep], v[keep])),
                      shape=(nn, nn)).tocsr()
    G = ((G + G.T) > 0).astype(np.int8).tocsr()
    G.sort_indices()
    return G


def overlapping_subdomains(G: sp.csr_matrix, part: np.ndarray, n_parts: int,
                           overlap: int) -> list[np.ndarray]:
    """O2: Omega_i^0 = {v : part(v) = i}; Omega_i^{k+1} = Omega_i^k plus its
    graph neighbours; returns the sorted node sets Omega_i' = Omega_i^overlap.
    (The paper allows growth by mesh elements or by nodes; here by graph layers
    of nodes, which is the algebraic overlap its experiments use.)"""
    order = np.argsort(part, kind="stable")
    bounds = np.searchsorted(part[order], np.arange(n_parts + 1))
    out = []
    for i in range(n_parts):
        nodes = np.sort(order[bounds[i]:bounds[i + 1]])
        for _ in range(overlap):
            nb = G[nodes].indices
            nodes = np.union1d(nodes, nb)
        out.append(nodes.astype(np.int64))
    return out


def dofs_of(nodes: np.ndarray, dpn: int) -> np.ndarray:
    """Dofs of a sorted node set in ascending order (node-major)."""
    return (dpn * nodes[:, None] + np.arange(dpn)[None, :]).ravel()


def interface(G: sp.csr_matrix, part: np.ndarray):
    """O4: v is on the interface iff it has a neighbour u with part(u) < part(v);
    S(v) = {part(v)} together with the parts of those lower neighbours.

    (The paper defines Gamma geometrically for a nonoverlapping
    decomposition.  For a partition of a matrix graph this lower-id rule gives
    a one-layer interface with A_II block diagonal, as the paper requires for
    the extension.)  Returns (is_gamma[bool n_nodes], S dict node -> tuple)."""
    coo = G.tocoo()
    u, v = coo.row, coo.col
    lower = part[u] < part[v]
    nn = G.shape[0]
    is_g = np.zeros(nn, dtype=bool)
    is_g[v[lower]] = True
    S = {}
    for node in np.nonzero(is_g)[0]:
        S[int(node)] = {int(part[node])}
    for a, b in zip(u[lower], v[lower]):
        S[int(b)].add(int(part[a]))
    return is_g, {k: tuple(sorted(s)) for k, s in S.items()}


def interface_from_sharing(share_ptr: np.ndarray, share_sub: np.ndarray, part: np.ndarray):
    """O4 for a decomposition into subdomains of elements (Sec. III): S(v) is
    the set of subdomains whose elements contain node v, as given, and v is
    on the interface iff S(v) holds two or more subdomains.  Every S(v) must
    contain part(v).  Returns (is_gamma, S) as interface() does."""
    nn = len(share_ptr) - 1
    is_g = np.zeros(nn, dtype=bool)
    S = {}
    for v in range(nn):
        sv = tuple(sorted(set(int(q) for q in share_sub[share_ptr[v]:share_ptr[v + 1]])))
        if int(part[v]) not in sv:
            raise ValueError(f"node {v}: its own subdomain does not share it")
        if len(sv) >= 2:
            is_g[v] = True
            S[v] = sv
    return is_g, S


def components(G: sp.csr_matrix, is_g: np.ndarray, S: dict) -> list[np.ndarray]:
    """O5: group interface nodes by their set S, split every group into
    connected pieces of the graph restricted to the group, and order the
    pieces by their smallest node id.  The pieces are disjoint (the paper
    allows overlapping pieces; with disjoint ones the partition of unity of
    O6 is the identity)."""
    groups: dict[tuple, list[int]] = {}
    for node in np.nonzero(is_g)[0]:
        groups.setdefault(S[int(node)], []).append(int(node))
    comps = []
    for key, nodes in groups.items():
        nodes = np.array(sorted(nodes), dtype=np.int64)
        sub = G[nodes][:, nodes]
        ncc, lab = csgraph.connected_components(sub, directed=False)
        for c in range(ncc):
            comps.append(nodes[lab == c])
    comps.sort(key=lambda c: int(c[0]))
    return comps


# ---------------------------------------------------------------------------
# O7-O8: interface coarse basis
# ---------------------------------------------------------------------------

def orthonormal_span(B: np.ndarray, drop_tol: float = 1e-10) -> np.ndarray:
    """O8: modified Gram-Schmidt with one reorthogonalisation pass; column j
    is dropped when what is left of it after projection has norm at most
    drop_tol times its original norm (or it is zero).  Returns the kept
    orthonormal columns in order.  (The paper only asks for a basis that
    spans the restricted null space; the span, and so M, does not depend on
    the basis chosen.)"""
    Q = []
    for j in range(B.shape[1]):
        bj = B[:, j].astype(np.float64)
        nb = np.linalg.norm(bj)
        if nb == 0.0:
            continue
        v = bj.copy()
        for _ in range(2):
            for q in Q:
                v -= (q @ v) * q
        nv = np.linalg.norm(v)
        if nv <= drop_tol * nb:
            continue
        Q.append(v / nv)
    if not Q:
        return np.zeros((B.shape[0], 0))
    return np.stack(Q, axis=1)


def rgdsw_coarse_nodes(comps: list, S: dict):
    """O8r (reduced GDSW, Sec. III: coarse functions only for vertices; the
    construction is only cited there).  Reading: component d is an ancestor
    of component c when S(c) is a proper subset of S(d); the coarse nodes
    are the components without an ancestor (with a 27-point coupling on a
    box partition: the cross points of the subdomains).  A coarse node
    belongs to itself; any other component belongs to the coarse nodes that
    are its ancestors.  Returns (coarse node list, owners per component),
    both ascending."""
    sets = [frozenset(S[int(c[0])]) for c in comps]
    coarse = [i for i, s in enumerate(sets) if not any(s < t for t in sets)]
    is_coarse = set(coarse)
    owners = []
    for i, s in enumerate(sets):
        owners.append([i] if i in is_coarse else [v for v in coarse if s < sets[v]])
    return coarse, owners


def rgdsw_weight(owners_of_component: list) -> float:
    """O8r: the weight of a component's rows in each coarse function it
    belongs to: 1 / (number of coarse nodes it belongs to), so that the
    weights of every interface node add up to one."""
    return 1.0 / len(owners_of_component)


def rgdsw_interface_basis(comps: list, S: dict, Z: np.ndarray, dpn: int, n: int):
    """O8r: the interface values of the coarse functions of every coarse node
    v: the null space Z on the components v belongs to, each component's rows
    weighted by 1 / (number of coarse nodes it belongs to) (a partition of
    unity on the interface), orthonormalised over that support as in O8.
    Columns ordered by coarse node.  Returns (Phi_Gamma as n x n0 CSR, the
    coarse columns touching each component, n0)."""
    coarse, owners = rgdsw_coarse_nodes(comps, S)
    support = {v: [] for v in coarse}
    for i, own in enumerate(owners):
        for v in own:
            support[v].append(i)
    comp_cols = [[] for _ in comps]
    rows, cols, vals = [], [], []
    n0 = 0
    for v in coarse:
        dofs = np.concatenate([dofs_of(comps[i], dpn) for i in support[v]])
        w = np.concatenate([np.full(comps[i].size * dpn, rgdsw_weight(owners[i])) for i in support[v]])
        Q = orthonormal_span(w[:, None] * Z[dofs, :])
        k = Q.shape[1]
        for i in support[v]:
            comp_cols[i].extend(range(n0, n0 + k))
        if k:
            rr, cc = np.meshgrid(dofs, np.arange(n0, n0 + k), indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(Q.ravel())
        n0 += k
    if rows:
        phi_g = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n0))
    else:
        phi_g = sp.csr_matrix((n, max(n0, 0)))
    return phi_g, comp_cols, n0


@dataclass
class CoarseSpace:
    comps: list            # node arrays
    comp_cols: list        # per component: the coarse columns that touch it
    phi: sp.csr_matrix     # n x n0
    n0: int


def extension_solve(Aii: sp.csc_matrix, rhs: np.ndarray) -> np.ndarray:
    """O9: A_{I_i I_i}^{-1} rhs by a sparse direct solve (a library primitive;
    the paper always uses a direct solver for the extension, Table IV note)."""
    return spla.splu(Aii).solve(rhs)


# ---------------------------------------------------------------------------
# the preconditioner
# ---------------------------------------------------------------------------

class GDSW:
    """The two-level additive Schwarz preconditioner of eq. (1) with the GDSW
    coarse space of eq. (2), built plainly in FP64.

    local = "exact" uses a sparse direct solve of every A_i; local = "ilu0"
    uses ILU(k) (k = ``ilu_level``, 0 by default) of A_i in its natural
    (ascending global dof) order with the two triangular solves replaced by
    ``sweeps`` undamped Jacobi sweeps each, from a zero start; the factors
    are exact ILU(k) factors, or with ``factor_sweeps`` > 0 the FastILU
    approximation after that many sweeps.  coarse = False drops the coarse
    term (one level); coarse_space = "rgdsw" takes the reduced GDSW interface
    basis of O8r instead of one block per component (O8).  sharing =
    (share_ptr, share_sub) takes the interface from the sets of subdomains
    sharing each node (interface_from_sharing) instead of the node graph.
    """

    def __init__(self, A, part, dpn: int, n_parts: int, Z=None, overlap: int = 1,
                 coarse: bool = True, local: str = "exact", sweeps: int = 5,
                 ilu_level: int = 0, factor_sweeps: int = 0, coarse_space: str = "gdsw", sharing=None):
        if coarse_space not in ("gdsw", "rgdsw"):
            raise ValueError(coarse_space)
        self.sharing = sharing
        self.coarse_space = coarse_space
        self.A = sp.csr_matrix(A, dtype=np.float64)
        self.A.sort_indices()
        self.n = self.A.shape[0]
        self.dpn = int(dpn)
        self.part = np.asarray(part, dtype=np.int64)
        self.n_parts = int(n_parts)
        self.overlap = int(overlap)
        self.local = local
        self.sweeps = int(sweeps)
        self.ilu_level = int(ilu_level)
        self.factor_sweeps = int(factor_sweeps)
        self.use_coarse = bool(coarse)
        if Z is None:
            Z = np.ones((self.n, 1))
        self.Z = np.asarray(Z, dtype=np.float64).reshape(self.n, -1)
        self._symbolic()
        self._local_factors()
        if self.use_coarse:
            self._coarse()
        else:
            self.cs = None

    # -- O1-O5 -------------------------------------------------------------
    def _symbolic(self):
        self.G = node_graph(self.A, self.dpn)
        self.ov_nodes = overlapping_subdomains(self.G, self.part, self.n_parts, self.overlap)
        self.R = [dofs_of(nd, self.dpn) for nd in self.ov_nodes]
        if self.sharing is None:
            self.is_gamma, self.S = interface(self.G, self.part)
        else:
            self.is_gamma, self.S = interface_from_sharing(self.sharing[0], self.sharing[1], self.part)
        self.comps = components(self.G, self.is_gamma, self.S)

    # -- O3, O11 -----------------------------------------------------------
    def _local_factors(self):
        self.local_solvers = []
        for Ri in self.R:
            if Ri.size == 0:
                # a subdomain id that owns no node: its term of eq. (1) is empty
                self.local_solvers.append(None)
                continue
            Ai = self.A[Ri][:, Ri].tocsr()
            Ai.sort_indices()
            if self.local == "exact":
                self.local_solvers.append(spla.splu(Ai.tocsc()))
            elif self.local == "ilu0":
                if self.ilu_level == 0 and self.factor_sweeps == 0:
                    self.local_solvers.append(ilu0_factors(Ai))
                else:
                    self.local_solvers.append(ilu_factors(Ai, self.ilu_level, self.factor_sweeps))
            else:
                raise ValueError(self.local)

    # -- O6-O10, O12 ---------------------------------------------------------
    def _coarse(self):
        dpn = self.dpn
        if self.coarse_space == "rgdsw":
            phi_g, comp_cols, n0 = rgdsw_interface_basis(self.comps, self.S, self.Z, dpn, self.n)
        else:
            rows, cols, vals = [], [], []
            comp_cols = []
            n0 = 0
            for c in self.comps:
                dofs = dofs_of(c, dpn)
                Q = orthonormal_span(self.Z[dofs, :])
                k = Q.shape[1]
                comp_cols.append(list(range(n0, n0 + k)))
                if k:
                    rr, cc = np.meshgrid(dofs, np.arange(n0, n0 + k), indexing="ij")
                    rows.append(rr.ravel())
                    cols.append(cc.ravel())
                    vals.append(Q.ravel())
                n0 += k
            if n0:
                phi_g = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                      shape=(self.n, n0))
        self.n0 = n0
        if n0 == 0:
            self.cs = None
            return
        gamma_dofs = dofs_of(np.nonzero(self.is_gamma)[0], dpn)
        interior_nodes = np.nonzero(~self.is_gamma)[0]
        # O9: Phi(I_i, :) = -A_{I_i I_i}^{-1} A_{I_i Gamma} Phi_Gamma per subdomain
        A_gamma_cols = self.A[:, gamma_dofs].tocsr()
        phi_g_rows = phi_g[gamma_dofs].tocsc()
        rows, cols, vals = [], [], []
        for i in range(self.n_parts):
            Ii = dofs_of(interior_nodes[self.part[interior_nodes] == i], dpn)
            if Ii.size == 0:
                continue
            Aii = self.A[Ii][:, Ii].tocsc()
            rhs = -(A_gamma_cols[Ii] @ phi_g_rows)          # sparse n_Ii x n0
            rhs = rhs.tocsc()
            used = np.nonzero(np.diff(rhs.indptr))[0]
            if used.size == 0:
                continue
            X = extension_solve(Aii, rhs[:, used].toarray())
            rr, cc = np.meshgrid(Ii, used, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(X.ravel())
        if rows:
            phi_i = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                  shape=(self.n, n0))
            phi = (phi_g + phi_i).tocsr()
        else:
            phi = phi_g.tocsr()
        phi.sort_indices()
        self.cs = CoarseSpace(self.comps, comp_cols, phi, n0)
        # O10
        A0 = (phi.T @ (self.A @ phi)).toarray()
        self.A0 = A0
        # O12
        self.A0_chol = sla.cho_factor(A0, lower=True)

    # -- O13 -------------------------------------------------------------------
    def local_solve(self, i: int, ri: np.ndarray) -> np.ndarray:
        f = self.local_solvers[i]
        if self.local == "exact":
            return f.solve(ri)
        return ilu0_jacobi_solve(f, ri, self.sweeps)

    def apply(self, r: np.ndarray) -> np.ndarray:
        """z = M^{-1} r, eq. (1): the one-level part over i = 1..n_p in
        ascending order, then the coarse part."""
        r = np.asarray(r, dtype=np.float64)
        z = np.zeros(self.n)
        for i, Ri in enumerate(self.R):
            if Ri.size:
                z[Ri] += self.local_solve(i, r[Ri])
        if self.cs is not None:
            r0 = self.cs.phi.T @ r
            z0 = sla.cho_solve(self.A0_chol, r0)
            z += self.cs.phi @ z0
        return z

    def coarse_apply(self, r: np.ndarray) -> np.ndarray:
        """The coarse term alone, Phi A_0^{-1} Phi^T r."""
        if self.cs is None:
            return np.zeros(self.n)
        return self.cs.phi @ sla.cho_solve(self.A0_chol, self.cs.phi.T @ r)

    # -- maps exported for bit-exact comparison ---------------------------------
    def maps(self) -> dict:
        ov_ptr = np.zeros(self.n_parts + 1, dtype=np.int64)
        ov_ptr[1:] = np.cumsum([r.size for r in self.R])
        comp_of = np.full(self.A.shape[0] // self.dpn, -1, dtype=np.int32)
        for c, nodes in enumerate(self.comps):
            comp_of[nodes] = c
        return {
            "ov_ptr": ov_ptr,
            "ov_idx": np.concatenate(self.R).astype(np.int64) if self.R else np.zeros(0, np.int64),
            "is_gamma": self.is_gamma.astype(np.int8),
            "comp_of_node": comp_of,
            "n_comp": len(self.comps),
            "n0": getattr(self, "n0", 0),
            "comp_rank": np.array([len(cc) for cc in self.cs.comp_cols], dtype=np.int32)
            if self.cs is not None else np.zeros(0, np.int32),
        }


# ---------------------------------------------------------------------------
# ILU(0) factors and the Jacobi-sweep triangular solves
# ---------------------------------------------------------------------------

@dataclass
class ILU0:
    NL: sp.csr_matrix      # strictly lower part of the unit-lower L
    NU: sp.csr_matrix      # strictly upper part of U
    d: np.ndarray          # diagonal of U


def ilu0_factors(Ai: sp.csr_matrix) -> ILU0:
    """ILU(0) of A_i on its own pattern, rows in the given order (plain C)."""
    M = sp.csr_matrix(Ai, dtype=np.float64, copy=True)
    M.sort_indices()
    rowptr = np.ascontiguousarray(M.indptr, dtype=np.int64)
    col = np.ascontiguousarray(M.indices, dtype=np.int32)
    val = np.ascontiguousarray(M.data, dtype=np.float64)
    rc = _lib().oracle_ilu0(M.shape[0], rowptr.ctypes.data, col.ctypes.data, val.ctypes.data)
    if rc != 0:
        raise np.linalg.LinAlgError(f"ILU(0) breakdown (code {rc})")
    F = sp.csr_matrix((val, col, rowptr), shape=M.shape)
    NL = sp.tril(F, k=-1, format="csr")
    NU = sp.triu(F, k=1, format="csr")
    return ILU0(NL, NU, F.diagonal().copy())


def iluk_pattern(Ai: sp.csr_matrix, level: int):
    """The ILU(level) pattern of A_i (level-of-fill rule, plain C): returns
    the CSR matrix holding A_i's values on that pattern (0 at fill entries)
    and the level of every entry."""
    M = sp.csr_matrix(Ai, dtype=np.float64, copy=True)
    M.sort_indices()
    n = M.shape[0]
    rowptr = np.ascontiguousarray(M.indptr, dtype=np.int64)
    col = np.ascontiguousarray(M.indices, dtype=np.int32)
    cap = max(4 * col.size, 16)
    while True:
        orp = np.zeros(n + 1, dtype=np.int64)
        oc = np.zeros(cap, dtype=np.int32)
        ol = np.zeros(cap, dtype=np.int32)
        nnz = _lib().oracle_iluk_pattern(n, rowptr.ctypes.data, col.ctypes.data, int(level),
                                         orp.ctypes.data, oc.ctypes.data, ol.ctypes.data, cap)
        if nnz == -2:
            raise MemoryError("ILU(k) pattern")
        if nnz >= 0:
            break
        cap = -nnz
    oc, ol = oc[:nnz], ol[:nnz]
    P = sp.csr_matrix((np.ones(nnz), oc, orp), shape=M.shape)
    # A's values on the pattern: positions of A's entries inside it
    vals = np.zeros(nnz)
    for i in range(n):
        cols = oc[orp[i]:orp[i + 1]]
        k = np.searchsorted(cols, col[rowptr[i]:rowptr[i + 1]])
        vals[orp[i] + k] = M.data[rowptr[i]:rowptr[i + 1]]
    P.data = vals
    return P, ol


def fastilu_sweeps(P: sp.csr_matrix, sweeps: int) -> sp.csr_matrix:
    """FastILU: the incomplete factors on the pattern of P (which holds the
    values a_ij of A there, 0 at fill) approximated by Jacobi sweeps over
    the factor entries (Sec. V-B, iterative variants).  Every sweep computes
    each entry from the previous sweep's values:
        i > j:  l_ij = (a_ij - sum_{m<j} l_im u_mj) / u_jj
        i <= j: u_ij =  a_ij - sum_{m<i} l_im u_mj
    (sums over the m with (i, m) and (m, j) in the pattern, ascending m).
    Start (a reading; the paper names no initial guess): l_ij = a_ij / a_jj,
    u_ij = a_ij, i.e. the lower and upper parts of A.  The result holds the
    strictly lower entries of the unit-lower L and the entries of U."""
    n = P.shape[0]
    ip, ix, a = P.indptr, P.indices, P.data
    where = [dict(zip(ix[ip[i]:ip[i + 1]].tolist(), range(ip[i], ip[i + 1]))) for i in range(n)]
    dpos = np.array([where[i][i] for i in range(n)])
    v = a.copy()
    for i in range(n):
        for e in range(ip[i], ip[i + 1]):
            if ix[e] < i:
                v[e] = a[e] / a[dpos[ix[e]]]
    for _ in range(sweeps):
        new = np.empty_like(v)
        for i in range(n):
            for e in range(ip[i], ip[i + 1]):
                j = int(ix[e])
                lim = min(i, j)
                acc = a[e]
                for f in range(ip[i], ip[i + 1]):
                    m = int(ix[f])
                    if m >= lim:
                        break
                    g = where[m].get(j)
                    if g is not None:
                        acc -= v[f] * v[g]
                new[e] = acc / v[dpos[j]] if i > j else acc
        v = new
    return sp.csr_matrix((v, ix.copy(), ip.copy()), shape=P.shape)


def ilu_factors(Ai: sp.csr_matrix, level: int = 0, factor_sweeps: int = 0) -> ILU0:
    """ILU(level) of A_i, rows in the given order: exact (row by row, plain
    C) when factor_sweeps == 0, else FastILU after factor_sweeps sweeps."""
    P, _ = iluk_pattern(Ai, level)
    if factor_sweeps > 0:
        F = fastilu_sweeps(P, factor_sweeps)
    else:
        rowptr = np.ascontiguousarray(P.indptr, dtype=np.int64)
        col = np.ascontiguousarray(P.indices, dtype=np.int32)
        val = np.ascontiguousarray(P.data, dtype=np.float64)
        rc = _lib().oracle_ilu0(P.shape[0], rowptr.ctypes.data, col.ctypes.data, val.ctypes.data)
        if rc != 0:
            raise np.linalg.LinAlgError(f"ILU({level}) breakdown (code {rc})")
        F = sp.csr_matrix((val, col, rowptr), shape=P.shape)
    NL = sp.tril(F, k=-1, format="csr")
    NU = sp.triu(F, k=1, format="csr")
    return ILU0(NL, NU, F.diagonal().copy())


def ilu0_jacobi_solve(f: ILU0, r: np.ndarray, sweeps: int) -> np.ndarray:
    """Approximate (LU)^{-1} r by Jacobi sweeps on each triangle:
    y^0 = 0, y^{k+1} = r - N_L y^k;  w^0 = 0, w^{k+1} = D_U^{-1}(y^K - N_U w^k).
    (Undamped, from a zero start; the paper's default is five sweeps each.)"""
    y = np.zeros_like(r)
    for _ in range(sweeps):
        y = r - f.NL @ y
    w = np.zeros_like(r)
    for _ in range(sweeps):
        w = (y - f.NU @ w) / f.d
    return w


# ---------------------------------------------------------------------------
# O14: Krylov solvers
# ---------------------------------------------------------------------------

@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    converged: bool
    rel_res_recursive: float
    rel_res_true: float
    history: list


def pcg(A, b, M=None, rtol: float = 1e-8, maxit: int = 1000,
        fixed_iters: int | None = None) -> SolveResult:
    """Preconditioned CG from x0 = 0.  Stops at the first k with
    ||r_k||_2 <= rtol ||b||_2 on the recursively updated residual (or after
    exactly ``fixed_iters`` iterations when given)."""
    A = sp.csr_matrix(A)
    b = np.asarray(b, dtype=np.float64)
    apply = (lambda v: v.copy()) if M is None else M.apply
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    hist = [1.0 if bnorm > 0 else 0.0]
    if bnorm == 0.0:
        return SolveResult(x, 0, True, 0.0, 0.0, hist)
    z = apply(r)
    p = z.copy()
    rho = r @ z
    k = 0
    converged = False
    limit = fixed_iters if fixed_iters is not None else maxit
    while k < limit:
        q = A @ p
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        k += 1
        rn = np.linalg.norm(r)
        hist.append(rn / bnorm)
        if fixed_iters is None and rn <= rtol * bnorm:
            converged = True
            break
        z = apply(r)
        rho_new = r @ z
        beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
    if fixed_iters is not None:
        converged = hist[-1] <= rtol
    true = np.linalg.norm(b - A @ x) / bnorm
    return SolveResult(x, k, converged, hist[-1], true, hist)


def gmres(A, b, M=None, rtol: float = 1e-8, restart: int = 30, maxit: int = 1000,
          fixed_iters: int | None = None) -> SolveResult:
    """Right-preconditioned restarted GMRES(m) from x0 = 0 with modified
    Gram-Schmidt Arnoldi and Givens rotations.  Stops when the Arnoldi
    residual estimate is <= rtol ||b||_2; the true residual is recomputed at
    every restart.  (The paper uses a single-reduce GMRES(30); in exact
    arithmetic it produces these same iterates.)"""
    A = sp.csr_matrix(A)
    b = np.asarray(b, dtype=np.float64)
    apply = (lambda v: v.copy()) if M is None else M.apply
    n = b.size
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = [1.0 if bnorm > 0 else 0.0]
    if bnorm == 0.0:
        return SolveResult(x, 0, True, 0.0, 0.0, hist)
    total = 0
    limit = fixed_iters if fixed_iters is not None else maxit
    converged = False
    while total < limit and not converged:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if fixed_iters is None and beta <= rtol * bnorm:
            converged = True
            break
        m = restart
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        Zs = []
        j_done = 0
        for j in range(m):
            zj = apply(V[:, j])
            Zs.append(zj)
            w = A @ zj
            for i in range(j + 1):
                H[i, j] = V[:, i] @ w
                w -= H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if fixed_iters is None and abs(g[j + 1]) <= rtol * bnorm:
                converged = True
                break
            if total >= limit:
                break
        y = sla.solve_triangular(H[:j_done, :j_done], g[:j_done])
        for i in range(j_done):
            x += y[i] * Zs[i]
    true = np.linalg.norm(b - A @ x) / bnorm
    if fixed_iters is not None:
        converged = true <= rtol
    return SolveResult(x, total, converged, hist[-1], true, hist)


# ---------------------------------------------------------------------------
# O14b single-reduce GMRES (Sec. VII: the experiments use a single-reduce
# variant of GMRES(30), one global reduction per iteration, cited there
# without its steps; reading: the classical Gram-Schmidt process applied
# twice, with the second pass and the normalisation of a basis vector
# delayed to the next step so that both share that step's one reduction.)
#
# Step j of a cycle holds Q = [q_0 .. q_{j-1}] (orthonormal), the columns
# 0 .. j-2 of the unrotated Hessenberg matrix H, the candidate u for q_j
# (already projected once against Q) with its first-pass coefficients a,
# and z = A M^{-1} u.  One reduction gives
#     c = Q^T u,  d = Q^T z,  e = u.u,  f = u.z.
# Then (Pythagoras, Q orthonormal) beta = sqrt(e - c.c) is the norm of the
# twice-projected candidate u - Q c, q_j = (u - Q c) / beta, and column j-1
# of H is (a + c; beta).  By linearity and the Arnoldi relation
# A M^{-1} Q = [Q q_j] H(0:j+1, 0:j),
#     A M^{-1} q_j = (z - [Q q_j] H c) / beta,
# whose projections onto Q and q_j follow from d, f and H c without touching
# the vectors again; subtracting them gives the next candidate.  Step 0 has
# Q empty and u = r, so its reduction also yields ||r||.
# ---------------------------------------------------------------------------

def sr_coefficients(H: np.ndarray, a_prev: np.ndarray, j: int, c: np.ndarray, d: np.ndarray,
                    e: float, f: float):
    """The small arithmetic of single-reduce step j: beta, the completed
    column j-1 of H (written into H when j >= 1), H c and the first-pass
    coefficients a of A M^{-1} q_j against q_0 .. q_j.  beta = 0 marks an
    invariant Krylov space (u already lies in the span of Q)."""
    beta2 = e - c @ c
    beta = float(np.sqrt(beta2)) if beta2 > 0.0 else 0.0
    if j >= 1:
        H[:j, j - 1] = a_prev + c
        H[j, j - 1] = beta
    if beta == 0.0:
        return beta, None, None
    Hc = H[:j + 1, :j] @ c
    a = np.empty(j + 1)
    a[:j] = (d - Hc[:j]) / beta
    a[j] = ((f - c @ d) / beta - Hc[j]) / beta
    return beta, Hc, a


def sr_basis_vector(Q: np.ndarray, j: int, u: np.ndarray, c: np.ndarray, beta: float) -> np.ndarray:
    """q_j = (u - Q c) / beta: the candidate's second projection and its
    normalisation."""
    return (u - Q[:, :j] @ c) / beta


def sr_next_candidate(Q: np.ndarray, j: int, z: np.ndarray, beta: float, Hc: np.ndarray,
                      a: np.ndarray) -> np.ndarray:
    """A M^{-1} q_j = (z - [Q q_j] H c) / beta, projected once against
    q_0 .. q_j with the coefficients a."""
    w = (z - Q[:, :j + 1] @ Hc) / beta
    return w - Q[:, :j + 1] @ a


def gmres_single_reduce(A, b, M=None, rtol: float = 1e-8, restart: int = 30, maxit: int = 1000,
                        fixed_iters: int | None = None, return_basis: bool = False):
    """Right-preconditioned restarted GMRES(m) from x0 = 0 with one global
    reduction per Arnoldi step (steps above).  In exact arithmetic it yields
    the iterates of ``gmres``.  Column j-1 of H is complete one step after
    A M^{-1} is applied to its candidate, so the residual estimate, the
    Givens rotations and the stopping test lag by one step; the last step of
    a cycle needs no operator application.  ``return_basis`` also returns
    (Q, H) of the last cycle (for checks of the Arnoldi relation)."""
    A = sp.csr_matrix(A)
    b = np.asarray(b, dtype=np.float64)
    apply = (lambda v: v.copy()) if M is None else M.apply
    n = b.size
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = [1.0 if bnorm > 0 else 0.0]
    basis = None
    if bnorm == 0.0:
        res = SolveResult(x, 0, True, 0.0, 0.0, hist)
        return (res, basis) if return_basis else res
    total = 0
    limit = fixed_iters if fixed_iters is not None else maxit
    converged = False
    while total < limit and not converged:
        m = restart
        Q = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        R = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        u = b - A @ x
        a = np.zeros(0)
        k = 0              # completed columns of this cycle
        stop = False
        for j in range(m + 1):
            z = A @ apply(u) if j < m else None
            c = Q[:, :j].T @ u
            e = u @ u
            d = Q[:, :j].T @ z if z is not None else np.zeros(j)
            f = u @ z if z is not None else 0.0
            beta, Hc, a_new = sr_coefficients(H, a, j, c, d, e, f)
            if j == 0:
                g[0] = beta
                if beta == 0.0 or (fixed_iters is None and beta <= rtol * bnorm):
                    converged = True
                    break
            else:
                # Givens rotations on the completed column j-1
                R[:j + 1, j - 1] = H[:j + 1, j - 1]
                for i in range(j - 1):
                    t = cs[i] * R[i, j - 1] + sn[i] * R[i + 1, j - 1]
                    R[i + 1, j - 1] = -sn[i] * R[i, j - 1] + cs[i] * R[i + 1, j - 1]
                    R[i, j - 1] = t
                den = np.hypot(R[j - 1, j - 1], R[j, j - 1])
                cs[j - 1] = R[j - 1, j - 1] / den
                sn[j - 1] = R[j, j - 1] / den
                R[j - 1, j - 1] = den
                R[j, j - 1] = 0.0
                g[j] = -sn[j - 1] * g[j - 1]
                g[j - 1] = cs[j - 1] * g[j - 1]
                total += 1
                k = j
                hist.append(abs(g[j]) / bnorm)
                if fixed_iters is None and abs(g[j]) <= rtol * bnorm:
                    converged = True
                    stop = True
                elif total >= limit:
                    stop = True
            if beta == 0.0:
                break
            Q[:, j] = sr_basis_vector(Q, j, u, c, beta)
            if stop or j == m:
                break
            u = sr_next_candidate(Q, j, z, beta, Hc, a_new)
            a = a_new
        if k > 0:
            y = sla.solve_triangular(R[:k, :k], g[:k])
            x += apply(Q[:, :k] @ y)
        basis = (Q[:, :k + 1].copy(), H[:k + 1, :k].copy())
        if k == 0:
            break
    true = np.linalg.norm(b - A @ x) / bnorm
    if fixed_iters is not None:
        converged = true <= rtol
    res = SolveResult(x, total, converged, hist[-1], true, hist)
    return (res, basis) if return_basis else res

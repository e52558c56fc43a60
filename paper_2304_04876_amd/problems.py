"""Seeded synthetic inputs for the GDSW preconditioner: matrices, partitions,
null spaces and right-hand sides.

This module only *builds inputs*.  It holds none of the preconditioner's
arithmetic (no overlap, interface, coarse basis, factorisation or Krylov
step), so both the independent CPU oracle and the GPU library's tests and
benchmarks draw their inputs from here.

Problems (the paper's experiments use 3D linear elasticity, Sec. VII; the
Poisson / diffusion workloads are the synthetic stand-ins used for the
throughput measurements):

* ``poisson3d(N)``: 7-point finite differences on the N^3 interior nodes of the
  unit cube, Dirichlet boundary eliminated, stencil (6, -1) with no h^2 scaling.
* ``diffusion3d(N, kappa)``: same stencil with a coefficient per primal cell;
  the coefficient of a grid edge is the mean of the four cells sharing it.
* ``elasticity_q1(Ne)``: trilinear hexahedra on a uniform Ne^3 mesh of the unit
  cube, 2x2x2 Gauss quadrature, isotropic material (E, nu), nodes on the x=0
  face clamped (eliminated), consistent load of a body force, dofs node-major.

Partitions are boxes: along each axis a node with grid index g (counting the
eliminated boundary layer) belongs to box ``min(g*P // G, P-1)`` where G is the
number of mesh cells along that axis.

Node numbering is lexicographic with x fastest.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class Problem:
    """A sparse SPD system with its box partition.

    A is a scipy CSR matrix with sorted column indices and float64 values.
    ``part[node]`` is the nonoverlapping subdomain of each node; ``dpn`` the
    number of dofs per node (dof = dpn*node + component).
    """
    name: str
    A: sp.csr_matrix
    part: np.ndarray          # int32 [n_nodes]
    dpn: int
    n_parts: int
    coords: np.ndarray        # float64 [n_nodes, 3]
    b: np.ndarray | None = None   # assembled load, if the problem defines one
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def n_nodes(self) -> int:
        return self.n // self.dpn


def _csr(rows, cols, vals, n) -> sp.csr_matrix:
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def box_index(g: np.ndarray, P: int, G: int) -> np.ndarray:
    """Box of grid index g along one axis: min(g*P // G, P-1)."""
    return np.minimum((g.astype(np.int64) * P) // G, P - 1).astype(np.int32)


def _box_partition_nodes(gx, gy, gz, P, Gx, Gy, Gz) -> np.ndarray:
    bx = box_index(gx, P[0], Gx)
    by = box_index(gy, P[1], Gy)
    bz = box_index(gz, P[2], Gz)
    return (bx + P[0] * (by + P[1] * bz)).astype(np.int32)


def _grid_edges_7pt(N: int):
    """Edges (u, v, axis, lower-node grid coords) between interior nodes of an
    N^3 grid, u < v, plus the grid coords of every node."""
    idx = np.arange(N ** 3, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    return idx, x, y, z


def poisson3d(N: int, P: int | tuple = 2) -> Problem:
    """7-point (6, -1) Laplacian on the N^3 interior nodes of the unit cube."""
    if isinstance(P, int):
        P = (P, P, P)
    n = N ** 3
    idx, x, y, z = _grid_edges_7pt(N)
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, 6.0)]
    for axis, coord, stride in ((0, x, 1), (1, y, N), (2, z, N * N)):
        m = coord < N - 1
        u = idx[m]
        v = u + stride
        rows += [u, v]
        cols += [v, u]
        vals += [np.full(u.size, -1.0), np.full(u.size, -1.0)]
    A = _csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)
    part = _box_partition_nodes(x + 1, y + 1, z + 1, P, N + 1, N + 1, N + 1)
    h = 1.0 / (N + 1)
    coords = np.stack([(x + 1) * h, (y + 1) * h, (z + 1) * h], axis=1)
    return Problem(f"poisson{N}^3_P{P[0]}x{P[1]}x{P[2]}", A, part, 1,
                   P[0] * P[1] * P[2], coords, meta={"N": N, "P": P})


def diffusion3d(N: int, kappa: np.ndarray, P: int | tuple = 2) -> Problem:
    """7-point FD for -div(kappa grad u) with kappa given per primal cell.

    ``kappa`` has (N+1)^3 entries (cells between grid nodes 0..N+1, x fastest).
    The coefficient on the edge between nodes (x,y,z) and (x+1,y,z) is the mean
    of the four cells that contain that edge; likewise for y and z edges.
    """
    if isinstance(P, int):
        P = (P, P, P)
    C = N + 1
    kap = np.asarray(kappa, dtype=np.float64).reshape(C, C, C)   # [cz, cy, cx]
    n = N ** 3
    idx, x, y, z = _grid_edges_7pt(N)
    gx, gy, gz = x + 1, y + 1, z + 1          # grid coords incl. boundary layer

    def edge_coef(axis, ax, ay, az):
        # lower node of the edge at grid coords (ax, ay, az); cells sharing it
        if axis == 0:
            c = (kap[az - 1, ay - 1, ax] + kap[az - 1, ay, ax] +
                 kap[az, ay - 1, ax] + kap[az, ay, ax])
        elif axis == 1:
            c = (kap[az - 1, ay, ax - 1] + kap[az - 1, ay, ax] +
                 kap[az, ay, ax - 1] + kap[az, ay, ax])
        else:
            c = (kap[az, ay - 1, ax - 1] + kap[az, ay - 1, ax] +
                 kap[az, ay, ax - 1] + kap[az, ay, ax])
        return 0.25 * c

    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for axis, coord, stride in ((0, x, 1), (1, y, N), (2, z, N * N)):
        # edge to the + neighbour (node with coord+1), lower node = this node
        cplus = edge_coef(axis, gx, gy, gz)
        # edge to the - neighbour, lower node = neighbour
        sh = [gx, gy, gz]
        sh = [s - (1 if a == axis else 0) for a, s in enumerate(sh)]
        cminus = edge_coef(axis, *sh)
        diag += cplus + cminus
        m = coord < N - 1
        u = idx[m]
        v = u + stride
        rows += [u, v]
        cols += [v, u]
        vals += [-cplus[m], -cplus[m]]
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    A = _csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)
    part = _box_partition_nodes(gx, gy, gz, P, N + 1, N + 1, N + 1)
    h = 1.0 / (N + 1)
    coords = np.stack([gx * h, gy * h, gz * h], axis=1)
    return Problem(f"diffusion{N}^3_P{P[0]}", A, part, 1, P[0] * P[1] * P[2],
                   coords, meta={"N": N, "P": P})


def q1_element_stiffness(h: float, E: float, nu: float) -> np.ndarray:
    """24x24 stiffness of a cubic trilinear element of side h (2x2x2 Gauss).

    Local node a = ax + 2*ay + 4*az (ax, ay, az in {0,1}); dofs 3*a + comp.
    """
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[3:, 3:] = np.eye(3) * mu
    gp = np.array([-1.0, 1.0]) / np.sqrt(3.0)
    sgn = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)]) * 2 - 1
    Ke = np.zeros((24, 24))
    detJ = (h / 2) ** 3
    for xi in gp:
        for eta in gp:
            for zeta in gp:
                q = np.array([xi, eta, zeta])
                dN = np.zeros((8, 3))
                for a in range(8):
                    f = 1 + sgn[a] * q
                    dN[a, 0] = sgn[a, 0] * f[1] * f[2] / 8
                    dN[a, 1] = f[0] * sgn[a, 1] * f[2] / 8
                    dN[a, 2] = f[0] * f[1] * sgn[a, 2] / 8
                dN *= 2.0 / h
                B = np.zeros((6, 24))
                for a in range(8):
                    gx, gy, gz = dN[a]
                    c = 3 * a
                    B[0, c] = gx
                    B[1, c + 1] = gy
                    B[2, c + 2] = gz
                    B[3, c] = gy
                    B[3, c + 1] = gx
                    B[4, c + 1] = gz
                    B[4, c + 2] = gy
                    B[5, c] = gz
                    B[5, c + 2] = gx
                Ke += B.T @ D @ B * detJ
    return 0.5 * (Ke + Ke.T)


def elasticity_q1(Ne: int, P: int | tuple = 2, E: float = 1.0, nu: float = 0.3,
                  body_force=(0.0, 0.0, -1.0)) -> Problem:
    """Q1 linear elasticity on [0,1]^3 with Ne^3 cubes, x=0 face clamped."""
    if isinstance(P, int):
        P = (P, P, P)
    M = Ne + 1
    h = 1.0 / Ne
    Ke = q1_element_stiffness(h, E, nu)
    # full-grid node id of each element's 8 corners
    e = np.arange(Ne ** 3, dtype=np.int64)
    ex, ey, ez = e % Ne, (e // Ne) % Ne, e // (Ne * Ne)
    corners = np.empty((e.size, 8), dtype=np.int64)
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        corners[:, a] = (ex + ax) + M * ((ey + ay) + M * (ez + az))
    # renumber: drop x=0 nodes, keep lexicographic order (x fastest)
    full = np.arange(M ** 3, dtype=np.int64)
    fx = full % M
    keep = fx > 0
    newid = np.full(M ** 3, -1, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()), dtype=np.int64)
    n_nodes = int(keep.sum())
    n = 3 * n_nodes
    cn = newid[corners]                              # -1 where clamped
    edof = (3 * cn[:, :, None] + np.arange(3)[None, None, :]).reshape(e.size, 24)
    edof[np.repeat(cn < 0, 3, axis=1)] = -1
    r = np.repeat(edof, 24, axis=1).ravel()
    c = np.tile(edof, (1, 24)).ravel()
    v = np.tile(Ke.ravel(), e.size)
    m = (r >= 0) & (c >= 0)
    A = _csr(r[m], c[m], v[m], n)
    A = ((A + A.T) * 0.5).tocsr()      # exact symmetry of the summed values
    A.sort_indices()
    # consistent load: each element gives h^3/8 * f to each of its 8 nodes
    b = np.zeros(n)
    w = h ** 3 / 8
    for comp in range(3):
        if body_force[comp] != 0.0:
            d = edof[:, comp::3].ravel()
            d = d[d >= 0]
            np.add.at(b, d, w * body_force[comp])
    gx, gy, gz = fx[keep], (full // M % M)[keep], (full // (M * M))[keep]
    part = _box_partition_nodes(gx, gy, gz, P, Ne, Ne, Ne)
    coords = np.stack([gx * h, gy * h, gz * h], axis=1).astype(np.float64)
    return Problem(f"elasticity_q1_{Ne}^3_P{P[0]}", A, part, 3, P[0] * P[1] * P[2],
                   coords, b=b, meta={"Ne": Ne, "P": P, "E": E, "nu": nu})


def element_sharing(prob: Problem):
    """For a Q1 mesh from elasticity_q1: the boxes of the elements around each
    node (the element decomposition that the node boxes come from: element
    (ex, ey, ez) lies in box (box_index(ex, P, Ne), ...)).  Returns the sets
    as (ptr int64 [n_nodes+1], boxes int32), ascending within each node."""
    Ne, P = prob.meta["Ne"], prob.meta["P"]
    h = 1.0 / Ne
    g = np.rint(prob.coords / h).astype(np.int64)            # grid index of each node
    nn = g.shape[0]
    cand = np.full((nn, 8), -1, dtype=np.int64)
    for a in range(8):
        d = np.array([a & 1, (a >> 1) & 1, (a >> 2) & 1]) - 1   # cells g-1 or g per axis
        c = g + d[None, :]
        ok = np.all((c >= 0) & (c <= Ne - 1), axis=1)
        bx = [np.minimum((c[:, k] * P[k]) // Ne, P[k] - 1) for k in range(3)]
        box = bx[0] + P[0] * (bx[1] + P[1] * bx[2])
        cand[ok, a] = box[ok]
    cand.sort(axis=1)
    keep = cand >= 0
    keep[:, 1:] &= cand[:, 1:] != cand[:, :-1]
    counts = keep.sum(axis=1)
    ptr = np.zeros(nn + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return ptr, cand[keep].astype(np.int32)


def constant_nullspace(prob: Problem) -> np.ndarray:
    """Null space of the Neumann operator of a scalar problem: one constant."""
    return np.ones((prob.n, 1))


def rigid_body_modes(prob: Problem) -> np.ndarray:
    """Three translations and three linearised rotations about the domain
    centre (0.5, 0.5, 0.5); n x 6, dofs node-major."""
    assert prob.dpn == 3
    nn = prob.n_nodes
    c = prob.coords - 0.5
    Z = np.zeros((prob.n, 6))
    for k in range(3):
        Z[k::3, k] = 1.0
    # rotation about z: (-y, x, 0); about x: (0, -z, y); about y: (z, 0, -x)
    Z[0::3, 3] = -c[:, 1]
    Z[1::3, 3] = c[:, 0]
    Z[1::3, 4] = -c[:, 2]
    Z[2::3, 4] = c[:, 1]
    Z[0::3, 5] = c[:, 2]
    Z[2::3, 5] = -c[:, 0]
    assert Z.shape[0] == 3 * nn
    return Z


def rhs_uniform(n: int, seed: int) -> np.ndarray:
    """Right-hand side uniform in (-1, 1) from a seeded generator."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def workload_poisson_small() -> Problem:
    """Poisson 20^3 interior grid, 2x2x2 boxes (exact local solves, CG)."""
    return poisson3d(20, 2)


def workload_poisson_large() -> Problem:
    """Poisson 128^3 (2,097,152 dofs), 8x8x8 = 512 boxes of 16^3 nodes."""
    return poisson3d(128, 8)


def workload_elasticity() -> Problem:
    """Q1 elasticity, 48^3 elements, 6x6x6 boxes of 8^3 elements."""
    return elasticity_q1(48, 6)


def batch_diffusion_specs(count: int = 256, seed: int = 2304):
    """Specs of the batch of independent diffusion problems: for problem k a
    generator from SeedSequence(seed).spawn(count)[k] draws, in this order,
    the grid edge N in [16, 48], the boxes per axis P in [2, 4], the cell
    coefficients exp(N(0,1)) on (N+1)^3 cells and the RHS uniform(-1,1)."""
    out = []
    for k, s in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(s)
        N = int(rng.integers(16, 49))
        P = int(rng.integers(2, 5))
        kappa = np.exp(rng.standard_normal((N + 1) ** 3))
        b = rng.uniform(-1.0, 1.0, N ** 3)
        out.append({"k": k, "N": N, "P": P, "kappa": kappa, "b": b})
    return out


def batch_diffusion_problem(spec) -> Problem:
    pr = diffusion3d(spec["N"], spec["kappa"], spec["P"])
    pr.b = spec["b"]
    return pr


SERVE_SIZES = (32, 41, 50, 59, 69, 78, 87, 96)


def serve_operator(N: int) -> Problem:
    """Resident Poisson operator of the serving stream: P = round(N/16)."""
    return poisson3d(N, int(round(N / 16)))

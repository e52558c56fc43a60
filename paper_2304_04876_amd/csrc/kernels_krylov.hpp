// Device kernels of the Krylov iteration (FP64): CSR SpMV, fused vector
// updates and dot products, for one or several independent problems packed
// in a handle, each with its own scalars and stopping test.  Every
// reduction is deterministic: fixed row blocks each write one partial (fixed
// tree within the workgroup), then one workgroup per problem sums its
// partials in index order and updates the problem's scalar state on the
// device, so the host only polls flags.  (The kernel boundary orders the
// partial writes before the final sum; no device-wide fences are needed.)
#pragma once

#include <cstddef>

#include "kernels_common.hpp"

namespace gdsw {

struct KState {
    double rho, sigma, alpha, beta, rr, bb, rtol2, red;
    int iters, done, status, fixed, maxit, pad;
};

enum { KS_RUNNING = 0, KS_CONVERGED = 1, KS_MAXIT = 2, KS_BREAKDOWN = 3, KS_IDLE = 4 };

constexpr int KNT = 256;
constexpr int KROWS = 256;    // rows per workgroup of the Krylov kernels (one row per thread)

// Row blocks of the Krylov kernels.  Block b covers rows [row0[b], row1[b])
// of problem prob[b]; the blocks of a problem are consecutive, so the
// partial sums of a problem, and the order they are added in, depend only on
// that problem: results are the same whether it is solved alone or packed
// with others.  A launch covers blocks base .. base + gridDim.x - 1.
struct KBlk {
    const int32_t *prob;
    const int32_t *row0;
    const int32_t *row1;
    int base;
};

// Sum of partials [lo, hi) in index order, by one workgroup.
__device__ __forceinline__ double sum_partials(const double *partial, int lo, int hi, double *sh) {
    // eight independent chains keep eight loads in flight per thread; the
    // order depends only on hi - lo
    constexpr int C = 8;
    double v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = 0.0;
    int q = lo + int(threadIdx.x);
    for (; q + (C - 1) * KNT < hi; q += C * KNT) {
        double a[C];
#pragma unroll
        for (int c = 0; c < C; ++c) a[c] = partial[q + c * KNT];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] += a[c];
    }
    for (; q < hi; q += KNT) v[0] += partial[q];
    const double t = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    return block_sum<double, KNT>(t, sh);
}

// A in sliced ELL form for the SpMV: slices of SELL_C consecutive rows, each
// slice padded to its longest row and stored slot-major, so that
// consecutive threads (rows) read consecutive addresses.  The columns are
// stored as 16-bit offsets from the row (dcol) when every entry lies within
// 32767 of the diagonal (banded orderings: the 7-point and the Q1 elasticity
// matrices here), else as 32-bit indices (col); the kernels take the form as
// a template argument D16.
constexpr int SELL_C = 256;
struct Sell {
    const int64_t *off;    // [nslices+1] value offsets of the slices
    const int32_t *width;  // [nslices] slots of each slice
    const double *val;
    const int32_t *col;    // 32-bit columns (null with dcol)
    const int16_t *dcol;   // column - row (null with col)
};

template <bool D16>
__device__ __forceinline__ int sell_col(const Sell &A, int i, int64_t e) {
    if constexpr (D16)
        return i + int(ld_once(&A.dcol[e]));
    else
        return ld_once(&A.col[e]);
}

template <bool D16>
__device__ __forceinline__ double sell_row(const Sell &A, int i, const double *__restrict__ x) {
    const int sl = i / SELL_C, lane = i % SELL_C;
    const int64_t base = A.off[sl] + lane;
    const int w = A.width[sl];
    // slots in chunks of 8: all loads of a chunk are issued before the
    // products are added (in slot order); slots past the slice's width
    // re-read its last slot (in bounds, no branch between the loads) and are
    // not added
    constexpr int U = 8;
    double acc = 0.0;
    for (int j0 = 0; j0 < w; j0 += U) {
        int c[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = base + int64_t(min(j0 + u, w - 1)) * SELL_C;
            c[u] = sell_col<D16>(A, i, e);
            v[u] = ld_once(&A.val[e]);
        }
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u < w) acc += v[u] * xv[u];
    }
    return acc;
}

// y = A x on n rows; with right-hand-side slots (n a multiple of the
// operator's dimension pn) row k pn + i of slot k is row i of A applied to
// slot k of x
template <bool D16>
__global__ __launch_bounds__(KNT) void k_spmv(Sell A, const double *__restrict__ x, double *__restrict__ y, int n,
                                              int pn) {
    const int i = blockIdx.x * KNT + threadIdx.x;
    if (i >= n) return;
    const int base = pn < n ? (i / pn) * pn : 0;
    y[i] = sell_row<D16>(A, i - base, x + base);
}

// One row of A (z + beta p_old): the vector is formed on the fly from z and
// the previous direction, the same fma for every occurrence of an entry, so
// the value a row uses for its neighbour equals the one that neighbour
// writes as its own p_new.
__device__ __forceinline__ double p_next(double beta, double pold, double z) { return __builtin_fma(beta, pold, z); }

template <bool D16>
__device__ __forceinline__ double sell_row_p(const Sell &A, int i, const double *__restrict__ z,
                                             const double *__restrict__ pold, double beta) {
    const int sl = i / SELL_C, lane = i % SELL_C;
    const int64_t base = A.off[sl] + lane;
    const int w = A.width[sl];
    constexpr int U = 8;
    double acc = 0.0;
    for (int j0 = 0; j0 < w; j0 += U) {
        int c[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {   // (as in sell_row)
            const int64_t e = base + int64_t(min(j0 + u, w - 1)) * SELL_C;
            c[u] = sell_col<D16>(A, i, e);
            v[u] = ld_once(&A.val[e]);
        }
        double zv[U], pv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            zv[u] = z[c[u]];
            pv[u] = pold[c[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u < w) acc += v[u] * p_next(beta, pv[u], zv[u]);
    }
    return acc;
}

// x = 0, r = b on the rows of the launched blocks
__global__ __launch_bounds__(KNT) void k_cg_init(double *__restrict__ x, double *__restrict__ r,
                                                 const double *__restrict__ b, KBlk kb) {
    const int blk = kb.base + blockIdx.x;
    for (int i = kb.row0[blk] + threadIdx.x; i < kb.row1[blk]; i += KNT) {
        x[i] = 0.0;
        r[i] = b[i];
    }
}

// The update p = z + beta p fused into the next product: p_new = z + beta
// p_old (written by each row for itself), q = A p_new and the partials of
// p_new . q.  At the start of CG p_old = z and beta = 0, so p_new = z.
template <bool D16>
__global__ __launch_bounds__(KNT) void k_cg_spmv_dot_p(Sell A, const double *__restrict__ z,
                                                       const double *__restrict__ pold, double *__restrict__ pnew,
                                                       double *__restrict__ q, double *__restrict__ partial,
                                                       const KState *st, KBlk kb, int pn) {
    const int blk = kb.base + blockIdx.x;
    const KState &S = st[kb.prob[blk]];
    if (S.done) return;
    __shared__ double sh[KNT / 64];
    const double beta = S.beta;
    // rows of right-hand-side slot k are k pn + i (a block never crosses a slot)
    const int row0 = kb.row0[blk];
    const int base = row0 >= pn ? (row0 / pn) * pn : 0;
    double dot = 0.0;
    for (int i = row0 + threadIdx.x; i < kb.row1[blk]; i += KNT) {
        const double acc = sell_row_p<D16>(A, i - base, z + base, pold + base, beta);
        const double pi = p_next(beta, pold[i], z[i]);
        pnew[i] = pi;
        __builtin_nontemporal_store(acc, &q[i]);   // (read once, by the update)
        dot += pi * acc;
    }
    dot = block_sum<double, KNT>(dot, sh);
    if (threadIdx.x == 0) partial[blk] = dot;
}

// The same for right-hand-side slots: one workgroup per row block of the
// operator takes that block in every slot, loading each matrix entry once
// for up to SG slots at a time (slot k's Krylov block is k nkb1 + b, its
// rows k pn + i).  Each slot's row sums, products and block partials are
// formed in the order of the one-slot kernel above, so the results are the
// same bits.
template <bool D16>
__global__ __launch_bounds__(KNT) void k_cg_spmv_dot_p_ms(Sell A, const double *__restrict__ z,
                                                          const double *__restrict__ pold, double *__restrict__ pnew,
                                                          double *__restrict__ q, double *__restrict__ partial,
                                                          const KState *st, KBlk kb, int pn, int ns, int nkb1) {
    constexpr int SG = 4, U = 8;
    __shared__ double sh[KNT / 64];
    const int b = blockIdx.x;
    const int row0 = kb.row0[b], row1 = kb.row1[b];
    for (int g0 = 0; g0 < ns; g0 += SG) {
        const int ng = min(SG, ns - g0);
        bool act[SG];
        double beta[SG], dot[SG];
        bool any = false;
#pragma unroll
        for (int j = 0; j < SG; ++j) {
            const KState *S = j < ng ? &st[kb.prob[(g0 + j) * nkb1 + b]] : nullptr;
            act[j] = S && !S->done;
            beta[j] = act[j] ? S->beta : 0.0;
            dot[j] = 0.0;
            any |= act[j];
        }
        if (!any) continue;   // (the whole workgroup)
        for (int i = row0 + threadIdx.x; i < row1; i += KNT) {
            const int sl = i / SELL_C, lane = i % SELL_C;
            const int64_t base = A.off[sl] + lane;
            const int w = A.width[sl];
            double acc[SG];
#pragma unroll
            for (int j = 0; j < SG; ++j) acc[j] = 0.0;
            for (int j0 = 0; j0 < w; j0 += U) {
                int c[U];
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {   // (as in sell_row)
                    const int64_t e = base + int64_t(min(j0 + u, w - 1)) * SELL_C;
                    c[u] = sell_col<D16>(A, i, e);
                    v[u] = ld_once(&A.val[e]);
                }
#pragma unroll
                for (int j = 0; j < SG; ++j) {
                    if (!act[j]) continue;
                    const int64_t so = int64_t(g0 + j) * pn;
                    double zv[U], pv[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        zv[u] = z[so + c[u]];
                        pv[u] = pold[so + c[u]];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (j0 + u < w) acc[j] += v[u] * p_next(beta[j], pv[u], zv[u]);
                }
            }
#pragma unroll
            for (int j = 0; j < SG; ++j) {
                if (!act[j]) continue;
                const int64_t o = int64_t(g0 + j) * pn + i;
                const double pi = p_next(beta[j], pold[o], z[o]);
                pnew[o] = pi;
                __builtin_nontemporal_store(acc[j], &q[o]);
                dot[j] += pi * acc[j];
            }
        }
#pragma unroll
        for (int j = 0; j < SG; ++j) {
            if (j >= ng) break;   // (uniform)
            const double t = block_sum<double, KNT>(dot[j], sh);
            if (threadIdx.x == 0 && act[j]) partial[(g0 + j) * nkb1 + b] = t;
        }
    }
}

// x += alpha p; r -= alpha q; partials of r.r (the stop test is taken
// together with beta after the apply)
__global__ __launch_bounds__(KNT) void k_cg_update_xr(double *__restrict__ x, double *__restrict__ r,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ q,
                                                      double *__restrict__ partial, const KState *st, KBlk kb) {
    const int blk = kb.base + blockIdx.x;
    const KState &S = st[kb.prob[blk]];
    if (S.done) return;
    __shared__ double sh[KNT / 64];
    const double alpha = S.alpha;
    double v = 0.0;
    for (int i = kb.row0[blk] + threadIdx.x; i < kb.row1[blk]; i += KNT) {
        // x and q are read once here (x again only in the next update)
        __builtin_nontemporal_store(ld_once(&x[i]) + alpha * p[i], &x[i]);
        const double ri = r[i] - alpha * ld_once(&q[i]);
        r[i] = ri;
        v += ri * ri;
    }
    v = block_sum<double, KNT>(v, sh);
    if (threadIdx.x == 0) partial[blk] = v;
}

// partials of a.b
__global__ __launch_bounds__(KNT) void k_dot(const double *__restrict__ a, const double *__restrict__ b,
                                             double *__restrict__ partial, const KState *st, int skip_if_done,
                                             KBlk kb) {
    const int blk = kb.base + blockIdx.x;
    if (skip_if_done && st[kb.prob[blk]].done) return;
    __shared__ double sh[KNT / 64];
    double v = 0.0;
    for (int i = kb.row0[blk] + threadIdx.x; i < kb.row1[blk]; i += KNT) v += a[i] * b[i];
    v = block_sum<double, KNT>(v, sh);
    if (threadIdx.x == 0) partial[blk] = v;
}

// rr = ||r||^2: iteration count and stop tests; returns whether CG stopped
__device__ __forceinline__ bool cg_rr_step(KState &S, double t) {
    S.rr = t;
    S.iters += 1;
    if (!isfinite(t)) {
        S.done = 1;
        S.status = KS_BREAKDOWN;
    } else if (S.fixed > 0) {
        if (S.iters >= S.fixed) {
            S.done = 1;
            S.status = (t <= S.rtol2 * S.bb) ? KS_CONVERGED : KS_MAXIT;
        }
    } else if (t <= S.rtol2 * S.bb) {
        S.done = 1;
        S.status = KS_CONVERGED;
    } else if (S.iters >= S.maxit) {
        S.done = 1;
        S.status = KS_MAXIT;
    }
    return S.done != 0;
}

// t = r.z of the new residual: beta = t / rho, rho = t
__device__ __forceinline__ void cg_beta_step(KState &S, double t) {
    if (!isfinite(t) || S.rho == 0.0) {
        S.done = 1;
        S.status = KS_BREAKDOWN;
    } else {
        S.beta = t / S.rho;
        S.rho = t;
    }
}

// One workgroup per problem (problems base .. base + gridDim.x - 1): total
// of its partials and the scalar step it feeds; kdone mirrors `done`.
enum {
    KF_BB = 0,      // bb = t
    KF_RHO = 1,     // rho = t
    KF_ALPHA = 2,   // sigma = t, alpha = rho / sigma
    KF_RR = 3,      // rr = t, iteration count and stop tests
    KF_BETA = 4,    // beta = t / rho, rho = t
    KF_RED = 5,     // red = t
    KF_RR_BETA = 6  // KF_RR with the total of partial2 (r.r), then KF_BETA with t (r.z)
};

// Totals of partials [lo, hi) of a and, if b != nullptr, of b, each in
// index order, by one workgroup of NT threads: eight independent chains per
// thread, so that a problem of up to 8 NT row blocks needs one round of
// loads; the order depends only on hi - lo.
template <int NT>
__device__ __forceinline__ void sum_partials_pair(const double *__restrict__ a, const double *__restrict__ b, int lo,
                                                  int hi, double *sh, double &ta, double &tb) {
    constexpr int C = 8;
    double va[C], vb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) va[c] = vb[c] = 0.0;
    int q = lo + int(threadIdx.x);
    for (; q + (C - 1) * NT < hi; q += C * NT) {
        double xa[C], xb[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            xa[c] = a[q + c * NT];
            xb[c] = b ? b[q + c * NT] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            va[c] += xa[c];
            vb[c] += xb[c];
        }
    }
    for (; q < hi; q += NT) {
        va[0] += a[q];
        if (b) vb[0] += b[q];
    }
    double sa = ((va[0] + va[1]) + (va[2] + va[3])) + ((va[4] + va[5]) + (va[6] + va[7]));
    double sb = ((vb[0] + vb[1]) + (vb[2] + vb[3])) + ((vb[4] + vb[5]) + (vb[6] + vb[7]));
    sa = wave_sum(sa);
    sb = wave_sum(sb);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        sh[w] = sa;
        sh[NT / 64 + w] = sb;
    }
    __syncthreads();
    ta = tb = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
        ta += sh[k];
        tb += sh[NT / 64 + k];
    }
}

constexpr int KFIN_NT = 1024;   // threads of k_cg_finish
__global__ __launch_bounds__(KFIN_NT) void k_cg_finish(const double *__restrict__ partial,
                                                       const int32_t *__restrict__ pb_ptr, KState *st,
                                                       int *__restrict__ kdone, int op, int base,
                                                       const double *__restrict__ partial2) {
    const int k = base + blockIdx.x;
    KState &S = st[k];
    if ((op == KF_ALPHA || op == KF_RR || op == KF_BETA || op == KF_RR_BETA) && S.done) return;
    __shared__ double sh[2 * KFIN_NT / 64];
    double t, t2;
    sum_partials_pair<KFIN_NT>(partial, op == KF_RR_BETA ? partial2 : nullptr, pb_ptr[k], pb_ptr[k + 1], sh, t, t2);
    if (op == KF_RR_BETA) {
        if (threadIdx.x != 0) return;
        if (!cg_rr_step(S, t2)) cg_beta_step(S, t);
        if (kdone) kdone[k] = S.done;
        return;
    }
    if (threadIdx.x != 0) return;
    switch (op) {
        case KF_BB:
            S.bb = t;
            if (t == 0.0) {   // zero right-hand side: x = 0 is the solution
                S.done = 1;
                S.status = KS_CONVERGED;
            } else if (!isfinite(t)) {
                S.done = 1;
                S.status = KS_BREAKDOWN;
            }
            break;
        case KF_RHO: S.rho = t; break;
        case KF_ALPHA:
            S.sigma = t;
            if (!(t > 0.0) || !isfinite(t)) {
                S.done = 1;
                S.status = KS_BREAKDOWN;
            } else {
                S.alpha = S.rho / t;
            }
            break;
        case KF_RR: cg_rr_step(S, t); break;
        case KF_BETA: cg_beta_step(S, t); break;
        default: S.red = t; break;
    }
    if (kdone) kdone[k] = S.done;
}

// p = z on the row blocks kb.base .. kb.base + nb - 1 (start of CG), UPB
// row blocks per workgroup
constexpr int UPB = 4;
static_assert(KROWS <= KNT, "one row per thread in a row block");
__global__ __launch_bounds__(KNT) void k_cg_start_p(double *__restrict__ p, const double *__restrict__ z, KBlk kb,
                                                    int nb) {
#pragma unroll
    for (int u = 0; u < UPB; ++u) {
        const int b = blockIdx.x * UPB + u;
        if (b >= nb) break;
        const int blk = kb.base + b;
        const int i = kb.row0[blk] + int(threadIdx.x);
        if (i < kb.row1[blk]) p[i] = z[i];
    }
}

// y = b - y
__global__ void k_residual(const double *__restrict__ b, double *__restrict__ y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = b[i] - y[i];
}

__global__ void k_copy(const double *__restrict__ a, double *__restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        b[i] = a[i];
}

}  // namespace gdsw

namespace gdsw {

// ---------------------------------------------------------------------------
// Restarted GMRES(m), right preconditioned, on the device.  The Arnoldi basis
// V ((m+1) x n, one vector after another), the Hessenberg matrix, the Givens
// rotations and the right-hand side g of the small least-squares problem live
// in device memory; the step index and stop flags are in GState, so the host
// only queues steps and polls once per chunk.  Orthogonalisation is classical
// Gram-Schmidt applied twice (two reductions per step instead of j+1).
constexpr int GM_MAX = 64;   // largest restart length
constexpr int GM_RED = 1024; // workgroups of the GMRES reductions (grid-stride rows)

struct GState {
    // the part the host polls (copied back up to `cs`)
    double bb, rtol2, beta, wnorm;
    int j;          // completed columns of the current cycle
    int total;      // Arnoldi steps overall
    int m, fixed, maxit;
    int cycle_done, done, status;
    double g[GM_MAX + 1];
    // device only
    double cs[GM_MAX], sn[GM_MAX], y[GM_MAX];
    double h[GM_MAX + 1];              // coefficients of the current projection
    double H[(GM_MAX + 1) * GM_MAX];   // column-major, leading dimension GM_MAX+1 (rotated columns)
    // single-reduce variant
    double Hu[(GM_MAX + 1) * GM_MAX];  // the same columns before the rotations
    double a[GM_MAX + 1];              // first-pass coefficients of the pending column
    double cc[GM_MAX], cg[GM_MAX + 1]; // coefficients of the vector update
    double inv_beta;
};
constexpr size_t GSTATE_POLL = offsetof(GState, cs);
constexpr int GM_LD = GM_MAX + 1;

// out[v] = sum over b < np of p[v * sv + b * sb], v < nv, by one workgroup:
// a wavefront takes VU values at a time, its lanes stride over b, then the
// wavefront's fixed tree; the order depends only on np.
template <int NT>
__device__ void sum_partial_values(const double *__restrict__ p, int64_t sv, int64_t sb, int np, int nv,
                                   double *out) {
    constexpr int NW = NT / 64, VU = 4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int v0 = wave * VU; v0 < nv; v0 += NW * VU) {
        double acc[VU];
#pragma unroll
        for (int u = 0; u < VU; ++u) acc[u] = 0.0;
        for (int b = lane; b < np; b += 64) {
            double t[VU];
#pragma unroll
            for (int u = 0; u < VU; ++u) t[u] = v0 + u < nv ? p[(v0 + u) * sv + b * sb] : 0.0;
#pragma unroll
            for (int u = 0; u < VU; ++u) acc[u] += t[u];
        }
#pragma unroll
        for (int u = 0; u < VU; ++u) {
            const double t = wave_sum(acc[u]);
            if (lane == 0 && v0 + u < nv) out[v0 + u] = t;
        }
    }
}

// w = A t (skipped once the cycle has stopped)
template <bool D16>
__global__ __launch_bounds__(KNT) void k_gm_spmv(Sell A, const double *__restrict__ t, double *__restrict__ w, int n,
                                                 const GState *st) {
    if (st->cycle_done) return;
    const int i = blockIdx.x * KNT + threadIdx.x;
    if (i >= n) return;
    w[i] = sell_row<D16>(A, i, t);
}

// v = V_j (j from the state), the vector the preconditioner is applied to
__global__ void k_gm_get(const double *__restrict__ V, double *__restrict__ v, int64_t n, const GState *st) {
    if (st->cycle_done) return;
    const double *src = V + int64_t(st->j) * n;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        v[i] = src[i];
}

// partials of h[i] = V_i . w for i <= j (one wavefront reduction per i)
__global__ __launch_bounds__(KNT) void k_gm_dots(const double *__restrict__ V, const double *__restrict__ w, int64_t n,
                                                 double *__restrict__ partial, const GState *st) {
    if (st->cycle_done) return;
    __shared__ double sh[(KNT / 64) * (GM_MAX + 1)];
    const int j = st->j;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = 0; i <= j; ++i) {
        const double *Vi = V + int64_t(i) * n;
        double a = 0.0;
        for (int64_t r = blockIdx.x * int64_t(KNT) + threadIdx.x; r < n; r += int64_t(gridDim.x) * KNT)
            a += Vi[r] * w[r];
        a = wave_sum(a);
        if (lane == 0) sh[wave * (GM_MAX + 1) + i] = a;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += KNT) {
        double t = 0.0;
        for (int q = 0; q < KNT / 64; ++q) t += sh[q * (GM_MAX + 1) + i];
        partial[int64_t(blockIdx.x) * (GM_MAX + 1) + i] = t;
    }
}

// h[i] = sum of the partials (index order); add = 1 adds into H(:, j)
constexpr int GM_FIN_NT = 1024;
__global__ __launch_bounds__(GM_FIN_NT) void k_gm_dots_finish(const double *__restrict__ partial, int np, GState *st,
                                                              int add) {
    if (st->cycle_done) return;
    __shared__ double sv[GM_MAX + 1];
    const int j = st->j;
    sum_partial_values<GM_FIN_NT>(partial, 1, GM_MAX + 1, np, j + 1, sv);
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += GM_FIN_NT) {
        const double t = sv[i];
        st->h[i] = t;
        if (add) st->H[j * (GM_MAX + 1) + i] += t;
        else st->H[j * (GM_MAX + 1) + i] = t;
    }
}

// w -= sum_{i <= j} h[i] V_i
__global__ void k_gm_subtract(const double *__restrict__ V, double *__restrict__ w, int64_t n, const GState *st) {
    if (st->cycle_done) return;
    const int j = st->j;
    for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < n; r += int64_t(gridDim.x) * blockDim.x) {
        double acc = w[r];
        for (int i = 0; i <= j; ++i) acc -= st->h[i] * V[int64_t(i) * n + r];
        w[r] = acc;
    }
}

// partials of ||w||^2 (skip: the cycle has stopped)
__global__ __launch_bounds__(KNT) void k_gm_sqnorm(const double *__restrict__ w, int64_t n,
                                                   double *__restrict__ partial, const GState *st, int at_start) {
    if (at_start ? st->done : st->cycle_done) return;
    __shared__ double sh[KNT / 64];
    double v = 0.0;
    for (int64_t r = blockIdx.x * int64_t(KNT) + threadIdx.x; r < n; r += int64_t(gridDim.x) * KNT) v += w[r] * w[r];
    v = block_sum<double, KNT>(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// finishes one Arnoldi step: H(j+1, j) = ||w||, the Givens rotations, g,
// the stop tests, and j += 1
__global__ __launch_bounds__(KNT) void k_gm_step_finish(const double *__restrict__ partial, int np, GState *st) {
    if (st->cycle_done) return;
    __shared__ double sh[KNT / 64];
    const double ss = sum_partials(partial, 0, np, sh);
    if (threadIdx.x != 0) return;
    const int j = st->j;
    double *Hj = st->H + j * (GM_MAX + 1);
    const double hn = sqrt(ss);
    Hj[j + 1] = hn;
    st->wnorm = hn;
    for (int i = 0; i < j; ++i) {
        const double t = st->cs[i] * Hj[i] + st->sn[i] * Hj[i + 1];
        Hj[i + 1] = -st->sn[i] * Hj[i] + st->cs[i] * Hj[i + 1];
        Hj[i] = t;
    }
    const double den = sqrt(Hj[j] * Hj[j] + Hj[j + 1] * Hj[j + 1]);
    if (!(den > 0.0) || !isfinite(den)) {
        st->cycle_done = 1;
        st->done = 1;
        st->status = KS_BREAKDOWN;
        return;
    }
    st->cs[j] = Hj[j] / den;
    st->sn[j] = Hj[j + 1] / den;
    Hj[j] = den;
    Hj[j + 1] = 0.0;
    st->g[j + 1] = -st->sn[j] * st->g[j];
    st->g[j] = st->cs[j] * st->g[j];
    st->j = j + 1;
    st->total += 1;
    const double res2 = st->g[j + 1] * st->g[j + 1];
    if (st->fixed > 0) {
        if (st->total >= st->fixed) { st->cycle_done = 1; st->done = 1; st->status = KS_CONVERGED; }
    } else if (res2 <= st->rtol2 * st->bb) {
        st->cycle_done = 1;
        st->done = 1;
        st->status = KS_CONVERGED;
    } else if (st->total >= st->maxit) {
        st->cycle_done = 1;
        st->done = 1;
        st->status = KS_MAXIT;
    }
    if (st->j >= st->m) st->cycle_done = 1;
    // a vanishing new direction: the cycle's Krylov space holds the solution
    if (hn == 0.0 && !st->cycle_done) st->cycle_done = 1;
}

// V_{j} = w / H(j, j-1)  (j already advanced)
__global__ void k_gm_scale(double *__restrict__ V, const double *__restrict__ w, int64_t n, const GState *st) {
    if (st->cycle_done || st->wnorm == 0.0) return;
    const double s = 1.0 / st->wnorm;
    double *dst = V + int64_t(st->j) * n;
    for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < n; r += int64_t(gridDim.x) * blockDim.x)
        dst[r] = w[r] * s;
}

// start of a cycle: beta = ||r|| (from the partials), stop tests,
// g = beta e_1, H = 0
__global__ __launch_bounds__(KNT) void k_gm_start_finish(const double *__restrict__ partial, int np, GState *st) {
    if (st->done) return;
    __shared__ double sh[KNT / 64];
    const double ss = sum_partials(partial, 0, np, sh);
    if (threadIdx.x != 0) return;
    st->beta = sqrt(ss);
    st->j = 0;
    for (int i = 0; i <= GM_MAX; ++i) st->g[i] = 0.0;
    for (int i = 0; i < (GM_MAX + 1) * GM_MAX; ++i) st->H[i] = 0.0;
    st->g[0] = st->beta;
    st->cycle_done = 0;
    if (!isfinite(ss)) {
        st->cycle_done = 1; st->done = 1; st->status = KS_BREAKDOWN;
    } else if (st->fixed <= 0 && ss <= st->rtol2 * st->bb) {
        st->cycle_done = 1; st->done = 1; st->status = KS_CONVERGED;
    } else if (st->fixed > 0 && st->total >= st->fixed) {
        st->cycle_done = 1; st->done = 1; st->status = KS_CONVERGED;
    } else if (ss == 0.0) {
        st->cycle_done = 1; st->done = 1; st->status = KS_CONVERGED;
    }
    st->wnorm = st->beta;
}

__global__ void k_gm_v0(double *__restrict__ V, const double *__restrict__ r, int64_t n, const GState *st) {
    if (st->done || st->beta == 0.0) return;
    const double s = 1.0 / st->beta;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        V[i] = r[i] * s;
}

// y = H(0:j, 0:j)^{-1} g(0:j) by back substitution (one thread)
__global__ void k_gm_lsq(GState *st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int j = st->j;
    for (int i = j - 1; i >= 0; --i) {
        double t = st->g[i];
        for (int k = i + 1; k < j; ++k) t -= st->H[k * (GM_MAX + 1) + i] * st->y[k];
        st->y[i] = t / st->H[i * (GM_MAX + 1) + i];
    }
}

// u = sum_{i < j} y_i V_i
__global__ void k_gm_combine(const double *__restrict__ V, double *__restrict__ u, int64_t n, const GState *st) {
    const int j = st->j;
    for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < n; r += int64_t(gridDim.x) * blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < j; ++i) acc += st->y[i] * V[int64_t(i) * n + r];
        u[r] = acc;
    }
}

// x += t
__global__ void k_add(double *__restrict__ x, const double *__restrict__ t, int64_t n) {
    for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < n; r += int64_t(gridDim.x) * blockDim.x)
        x[r] += t[r];
}

// ---------------------------------------------------------------------------
// Single-reduce GMRES(m) (Sec. VII: the experiments' Krylov solver performs
// one global reduction per iteration).  Classical Gram-Schmidt applied
// twice, with the second pass and the normalisation of each basis vector
// delayed to the next step so that both share its one reduction.  Step j
// holds Q = [q_0 .. q_{j-1}], the candidate u for q_j (projected once) and
// z = A M^{-1} u.  One reduction gives c = Q^T u, d = Q^T z, e = u.u,
// f = u.z; then beta = sqrt(e - c.c), q_j = (u - Q c) / beta, column j-1 of
// H = (a + c; beta), and, by the Arnoldi relation,
// A M^{-1} q_j = (z - [Q q_j] H c) / beta, whose projections a onto
// q_0 .. q_j follow from d, f and H c; the next candidate is
// A M^{-1} q_j - [Q q_j] a.  Step 0 has Q empty and u = r.

constexpr int SR_R = 4;          // rows per thread and chunk of the reduction
constexpr int SR_MAXB = 1024;    // workgroups of the reduction (chunks are strided over them)
constexpr int SR_NV = 2 * GM_MAX + 2;

// Partials of c_i (value i), d_i (j + i), e (2j), f (2j + 1), value-major:
// partial[v * SR_MAXB + block].  z == nullptr (the last step of a cycle):
// d and f are zero.
__global__ __launch_bounds__(KNT) void k_sr_reduce(const double *__restrict__ Q, const double *__restrict__ u,
                                                   const double *__restrict__ z, int64_t n, int j,
                                                   double *__restrict__ partial, const GState *st) {
    if (st->cycle_done) return;
    __shared__ double sh[KNT / 64][SR_NV];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nv = 2 * j + 2;
    for (int v = lane; v < nv; v += 64) sh[wave][v] = 0.0;
    const int64_t nchunk = (n + int64_t(KNT) * SR_R - 1) / (int64_t(KNT) * SR_R);
    for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        const int64_t r0 = ch * KNT * SR_R + threadIdx.x;
        double uu[SR_R], zz[SR_R];
#pragma unroll
        for (int k = 0; k < SR_R; ++k) {
            const int64_t r = r0 + int64_t(k) * KNT;
            uu[k] = r < n ? u[r] : 0.0;
            zz[k] = (z != nullptr && r < n) ? z[r] : 0.0;
        }
        double e = 0.0, f = 0.0;
#pragma unroll
        for (int k = 0; k < SR_R; ++k) {
            e += uu[k] * uu[k];
            f += uu[k] * zz[k];
        }
        e = wave_sum(e);
        f = wave_sum(f);
        if (lane == 0) {
            sh[wave][2 * j] += e;
            sh[wave][2 * j + 1] += f;
        }
        // four basis vectors at a time: all their loads are issued first
        constexpr int U = 4;
        int i = 0;
        for (; i + U <= j; i += U) {
            double q[U][SR_R];
#pragma unroll
            for (int t = 0; t < U; ++t)
#pragma unroll
                for (int k = 0; k < SR_R; ++k) {
                    const int64_t r = r0 + int64_t(k) * KNT;
                    q[t][k] = r < n ? Q[int64_t(i + t) * n + r] : 0.0;
                }
#pragma unroll
            for (int t = 0; t < U; ++t) {
                double c = 0.0, d = 0.0;
#pragma unroll
                for (int k = 0; k < SR_R; ++k) {
                    c += q[t][k] * uu[k];
                    d += q[t][k] * zz[k];
                }
                c = wave_sum(c);
                d = wave_sum(d);
                if (lane == 0) {
                    sh[wave][i + t] += c;
                    sh[wave][j + i + t] += d;
                }
            }
        }
        for (; i < j; ++i) {
            double c = 0.0, d = 0.0;
#pragma unroll
            for (int k = 0; k < SR_R; ++k) {
                const int64_t r = r0 + int64_t(k) * KNT;
                const double q = r < n ? Q[int64_t(i) * n + r] : 0.0;
                c += q * uu[k];
                d += q * zz[k];
            }
            c = wave_sum(c);
            d = wave_sum(d);
            if (lane == 0) {
                sh[wave][i] += c;
                sh[wave][j + i] += d;
            }
        }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += KNT) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < KNT / 64; ++w) t += sh[w][v];
        partial[int64_t(v) * SR_MAXB + blockIdx.x] = t;
    }
}

// The small arithmetic of step j (one workgroup): sums the partials,
// completes column j-1 of H, forms H c, the first-pass coefficients of the
// next column and the vector-update coefficients, then (one thread) the
// Givens rotation of column j-1, g and the stopping tests.
constexpr int SR_FIN_NT = 1024;
__global__ __launch_bounds__(SR_FIN_NT) void k_sr_finish(const double *__restrict__ partial, int np, GState *st,
                                                         int j) {
    if (st->cycle_done) return;
    __shared__ double sv[SR_NV];
    __shared__ double sH[GM_LD * GM_MAX];
    __shared__ double sHc[GM_MAX + 1], scs[GM_MAX], ssn[GM_MAX], sdot[2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    sum_partial_values<SR_FIN_NT>(partial, SR_MAXB, 1, np, 2 * j + 2, sv);
    // columns 0 .. j-2 (rows 0 .. j), the rotations so far
    for (int i = 0; i + 1 < j; ++i)
        for (int k = tid; k <= j; k += SR_FIN_NT) sH[k + i * GM_LD] = st->Hu[k + i * GM_LD];
    for (int i = tid; i + 1 < j; i += SR_FIN_NT) {
        scs[i] = st->cs[i];
        ssn[i] = st->sn[i];
    }
    __syncthreads();
    const double *c = sv, *d = sv + j;
    const double e = sv[2 * j], f = sv[2 * j + 1];
    if (wave == 0) {
        double cc = 0.0, cd = 0.0;
        for (int i = lane; i < j; i += 64) {
            cc += c[i] * c[i];
            cd += c[i] * d[i];
        }
        cc = wave_sum(cc);
        cd = wave_sum(cd);
        if (lane == 0) {
            sdot[0] = cc;
            sdot[1] = cd;
        }
    }
    for (int i = tid; i < j; i += SR_FIN_NT) sH[i + (j - 1) * GM_LD] = st->a[i] + c[i];
    __syncthreads();
    const double beta2 = e - sdot[0];
    const bool finite = isfinite(beta2) && isfinite(f);
    const double beta = beta2 > 0.0 && finite ? sqrt(beta2) : 0.0;
    if (j >= 1 && tid == 0) sH[j + (j - 1) * GM_LD] = beta;
    __syncthreads();
    if (j >= 1)
        for (int k = tid; k <= j; k += SR_FIN_NT) st->Hu[k + (j - 1) * GM_LD] = sH[k + (j - 1) * GM_LD];
    for (int k = tid; k <= j; k += SR_FIN_NT) {
        double t = 0.0;   // (H c)_k: column i has rows 0 .. i+1
        for (int i = k > 0 ? k - 1 : 0; i < j; ++i) t += sH[k + i * GM_LD] * c[i];
        sHc[k] = t;
    }
    __syncthreads();
    if (beta > 0.0) {
        const double ib = 1.0 / beta;
        for (int k = tid; k <= j; k += SR_FIN_NT) {
            const double a = k < j ? (d[k] - sHc[k]) * ib : ((f - sdot[1]) * ib - sHc[j]) * ib;
            st->a[k] = a;
            st->cg[k] = sHc[k] * ib + a;
            if (k < j) st->cc[k] = c[k];
        }
        if (tid == 0) st->inv_beta = ib;
    }
    if (tid != 0) return;
    if (!finite) {
        st->cycle_done = 1;
        st->done = 1;
        st->status = KS_BREAKDOWN;
        return;
    }
    if (j == 0) {
        // ||r|| of the cycle's start
        st->beta = beta;
        st->wnorm = beta;
        st->g[0] = beta;
        if (beta == 0.0 || (st->fixed <= 0 && beta2 <= st->rtol2 * st->bb) ||
            (st->fixed > 0 && st->total >= st->fixed)) {
            st->cycle_done = 1;
            st->done = 1;
            st->status = KS_CONVERGED;
        }
        return;
    }
    // Givens rotations on the completed column j-1
    double *x = sH + (j - 1) * GM_LD;
    for (int i = 0; i + 1 < j; ++i) {
        const double t = scs[i] * x[i] + ssn[i] * x[i + 1];
        x[i + 1] = -ssn[i] * x[i] + scs[i] * x[i + 1];
        x[i] = t;
    }
    const double den = sqrt(x[j - 1] * x[j - 1] + x[j] * x[j]);
    if (!(den > 0.0) || !isfinite(den)) {
        st->cycle_done = 1;
        st->done = 1;
        st->status = KS_BREAKDOWN;
        return;
    }
    const double cj = x[j - 1] / den, sj = x[j] / den;
    st->cs[j - 1] = cj;
    st->sn[j - 1] = sj;
    x[j - 1] = den;
    x[j] = 0.0;
    double *Rj = st->H + (j - 1) * GM_LD;
    for (int k = 0; k <= j; ++k) Rj[k] = x[k];
    const double gp = st->g[j - 1];
    st->g[j] = -sj * gp;
    st->g[j - 1] = cj * gp;
    st->j = j;
    st->total += 1;
    st->wnorm = beta;
    const double res2 = st->g[j] * st->g[j];
    if (st->fixed > 0) {
        if (st->total >= st->fixed) { st->cycle_done = 1; st->done = 1; st->status = KS_CONVERGED; }
    } else if (res2 <= st->rtol2 * st->bb) {
        st->cycle_done = 1;
        st->done = 1;
        st->status = KS_CONVERGED;
    } else if (st->total >= st->maxit) {
        st->cycle_done = 1;
        st->done = 1;
        st->status = KS_MAXIT;
    }
    if (j >= st->m) st->cycle_done = 1;
    // an invariant Krylov space: the cycle holds the solution
    if (beta == 0.0) st->cycle_done = 1;
}

// q_j = (u - Q c) / beta into column j of Q, and the next candidate
// u = z / beta - sum_{k <= j} cg_k q_k (the same pass over Q).
__global__ __launch_bounds__(256) void k_sr_update(double *__restrict__ Q, double *__restrict__ u,
                                                   const double *__restrict__ z, int64_t n, int j,
                                                   const GState *st) {
    if (st->cycle_done) return;
    const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (r >= n) return;
    double ac = 0.0, ag = 0.0;
    constexpr int U = 8;
    int i = 0;
    for (; i + U <= j; i += U) {
        double q[U];
#pragma unroll
        for (int t = 0; t < U; ++t) q[t] = Q[int64_t(i + t) * n + r];
#pragma unroll
        for (int t = 0; t < U; ++t) {
            ac += st->cc[i + t] * q[t];
            ag += st->cg[i + t] * q[t];
        }
    }
    for (; i < j; ++i) {
        const double q = Q[int64_t(i) * n + r];
        ac += st->cc[i] * q;
        ag += st->cg[i] * q;
    }
    const double ib = st->inv_beta;
    const double qj = (u[r] - ac) * ib;
    Q[int64_t(j) * n + r] = qj;
    u[r] = (z[r] * ib - ag) - st->cg[j] * qj;
}

// start of a single-reduce cycle: H, g and the step count cleared
__global__ void k_sr_cycle_start(GState *st) {
    if (st->done) return;
    for (int i = threadIdx.x; i < GM_LD * GM_MAX; i += blockDim.x) {
        st->H[i] = 0.0;
        st->Hu[i] = 0.0;
    }
    for (int i = threadIdx.x; i <= GM_MAX; i += blockDim.x) st->g[i] = 0.0;
    if (threadIdx.x == 0) {
        st->j = 0;
        st->cycle_done = 0;
    }
}

}  // namespace gdsw

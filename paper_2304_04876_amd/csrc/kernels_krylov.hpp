// Device kernels of the Krylov iteration (FP64): CSR SpMV, fused vector
// updates and dot products, for one or several independent problems packed
// in a handle, each with its own scalars and stopping test.  Every
// reduction is deterministic: fixed row blocks each write one partial (fixed
// tree within the workgroup), then one workgroup per problem sums its
// partials in index order and updates the problem's scalar state on the
// device, so the host only polls flags.  (The kernel boundary orders the
// partial writes before the final sum; no device-wide fences are needed.)
#pragma once

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
// consecutive threads (rows) read consecutive addresses.
constexpr int SELL_C = 256;
struct Sell {
    const int64_t *off;    // [nslices+1] value offsets of the slices
    const int32_t *width;  // [nslices] slots of each slice
    const double *val;
    const int32_t *col;
};

__device__ __forceinline__ double sell_row(const Sell &A, int i, const double *__restrict__ x) {
    const int sl = i / SELL_C, lane = i % SELL_C;
    const int64_t base = A.off[sl] + lane;
    const int w = A.width[sl];
    // slots in chunks of 8: all loads of a chunk are issued before the
    // products are added (in slot order)
    constexpr int U = 8;
    double acc = 0.0;
    for (int j0 = 0; j0 < w; j0 += U) {
        int c[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = base + int64_t(j0 + u) * SELL_C;
            c[u] = j0 + u < w ? A.col[e] : 0;
            v[u] = j0 + u < w ? A.val[e] : 0.0;
        }
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = j0 + u < w ? x[c[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + u < w) acc += v[u] * xv[u];
    }
    return acc;
}

__global__ __launch_bounds__(KNT) void k_spmv(Sell A, const double *__restrict__ x, double *__restrict__ y, int n) {
    const int i = blockIdx.x * KNT + threadIdx.x;
    if (i >= n) return;
    y[i] = sell_row(A, i, x);
}

// One row of A (z + beta p_old): the vector is formed on the fly from z and
// the previous direction, the same fma for every occurrence of an entry, so
// the value a row uses for its neighbour equals the one that neighbour
// writes as its own p_new.
__device__ __forceinline__ double p_next(double beta, double pold, double z) { return __builtin_fma(beta, pold, z); }

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
        for (int u = 0; u < U; ++u) {
            const int64_t e = base + int64_t(j0 + u) * SELL_C;
            c[u] = j0 + u < w ? A.col[e] : 0;
            v[u] = j0 + u < w ? A.val[e] : 0.0;
        }
        double zv[U], pv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            zv[u] = j0 + u < w ? z[c[u]] : 0.0;
            pv[u] = j0 + u < w ? pold[c[u]] : 0.0;
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
__global__ __launch_bounds__(KNT) void k_cg_spmv_dot_p(Sell A, const double *__restrict__ z,
                                                       const double *__restrict__ pold, double *__restrict__ pnew,
                                                       double *__restrict__ q, double *__restrict__ partial,
                                                       const KState *st, KBlk kb) {
    const int blk = kb.base + blockIdx.x;
    const KState &S = st[kb.prob[blk]];
    if (S.done) return;
    __shared__ double sh[KNT / 64];
    const double beta = S.beta;
    double dot = 0.0;
    for (int i = kb.row0[blk] + threadIdx.x; i < kb.row1[blk]; i += KNT) {
        const double acc = sell_row_p(A, i, z, pold, beta);
        const double pi = p_next(beta, pold[i], z[i]);
        pnew[i] = pi;
        q[i] = acc;
        dot += pi * acc;
    }
    dot = block_sum<double, KNT>(dot, sh);
    if (threadIdx.x == 0) partial[blk] = dot;
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
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
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

__global__ __launch_bounds__(KNT) void k_cg_finish(const double *__restrict__ partial, const int32_t *__restrict__ pb_ptr,
                                                   KState *st, int *__restrict__ kdone, int op, int base,
                                                   const double *__restrict__ partial2) {
    const int k = base + blockIdx.x;
    KState &S = st[k];
    if ((op == KF_ALPHA || op == KF_RR || op == KF_BETA || op == KF_RR_BETA) && S.done) return;
    __shared__ double sh[KNT / 64];
    double t = sum_partials(partial, pb_ptr[k], pb_ptr[k + 1], sh);
    if (op == KF_RR_BETA) {
        __syncthreads();   // sh is reused
        const double t2 = sum_partials(partial2, pb_ptr[k], pb_ptr[k + 1], sh);
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
    double H[(GM_MAX + 1) * GM_MAX];   // column-major, leading dimension GM_MAX+1
    double cs[GM_MAX], sn[GM_MAX], g[GM_MAX + 1], y[GM_MAX];
    double h[GM_MAX + 1];              // coefficients of the current projection
    double bb, rtol2, beta, wnorm;
    int j;          // columns of the current cycle so far
    int total;      // Arnoldi steps overall
    int m, fixed, maxit;
    int cycle_done, done, status;
};

// w = A t (skipped once the cycle has stopped)
__global__ __launch_bounds__(KNT) void k_gm_spmv(Sell A, const double *__restrict__ t, double *__restrict__ w, int n,
                                                 const GState *st) {
    if (st->cycle_done) return;
    const int i = blockIdx.x * KNT + threadIdx.x;
    if (i >= n) return;
    w[i] = sell_row(A, i, t);
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
__global__ __launch_bounds__(KNT) void k_gm_dots_finish(const double *__restrict__ partial, int np, GState *st,
                                                        int add) {
    if (st->cycle_done) return;
    const int j = st->j;
    for (int i = threadIdx.x; i <= j; i += KNT) {
        double t = 0.0;
        for (int b = 0; b < np; ++b) t += partial[int64_t(b) * (GM_MAX + 1) + i];
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

}  // namespace gdsw

// Device kernels of the Krylov iteration (FP64): CSR SpMV, fused vector
// updates and dot products.  Every reduction is deterministic: each
// workgroup writes a partial in a fixed order and the last workgroup to
// finish (found with a counter) sums the partials in index order, then
// updates the scalar state on the device, so the host only polls a flag.
#pragma once

#include "kernels_common.hpp"

namespace gdsw {

struct KState {
    double rho, sigma, alpha, beta, rr, bb, rtol2, red;
    int iters, done, status, fixed, maxit, pad;
    unsigned cnt[8];
};

enum { KS_RUNNING = 0, KS_CONVERGED = 1, KS_MAXIT = 2, KS_BREAKDOWN = 3 };

constexpr int KNT = 256;

// sums gridDim.x partials in index order; called by the last workgroup only
__device__ __forceinline__ double finish_partials(const double *partial, int np, double *sh) {
    double v = 0.0;
    for (int q = threadIdx.x; q < np; q += KNT) v += __builtin_nontemporal_load(partial + q);
    return block_sum<double, KNT>(v, sh);
}

// returns true in every thread of the last workgroup to arrive
__device__ __forceinline__ bool arrive_last(unsigned *cnt, bool *flag) {
    __threadfence();
    if (threadIdx.x == 0) *flag = (atomicAdd(cnt, 1u) == gridDim.x - 1);
    __syncthreads();
    const bool last = *flag;
    if (last) __threadfence();
    return last;
}

__global__ __launch_bounds__(KNT) void k_spmv(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                              const double *__restrict__ val, const double *__restrict__ x,
                                              double *__restrict__ y, int n) {
    const int i = blockIdx.x * KNT + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) acc += val[p] * x[col[p]];
    y[i] = acc;
}

// q = A p; sigma = p.q; alpha = rho / sigma
__global__ __launch_bounds__(KNT) void k_cg_spmv_dot(const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ p, double *__restrict__ q,
                                                     int n, double *__restrict__ partial, KState *st) {
    if (st->done) return;
    __shared__ double sh[KNT / 64];
    __shared__ bool last;
    const int i = blockIdx.x * KNT + threadIdx.x;
    double dot = 0.0;
    if (i < n) {
        double acc = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += val[k] * p[col[k]];
        q[i] = acc;
        dot = p[i] * acc;
    }
    dot = block_sum<double, KNT>(dot, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = dot;
    if (!arrive_last(&st->cnt[0], &last)) return;
    const double sigma = finish_partials(partial, gridDim.x, sh);
    if (threadIdx.x == 0) {
        st->cnt[0] = 0;
        st->sigma = sigma;
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            st->done = 1;
            st->status = KS_BREAKDOWN;
        } else {
            st->alpha = st->rho / sigma;
        }
    }
}

// x += alpha p; r -= alpha q; rr = r.r; convergence test
__global__ __launch_bounds__(KNT) void k_cg_update_xr(double *__restrict__ x, double *__restrict__ r,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ q, int n,
                                                      double *__restrict__ partial, KState *st) {
    if (st->done) return;
    __shared__ double sh[KNT / 64];
    __shared__ bool last;
    const double alpha = st->alpha;
    const int i = blockIdx.x * KNT + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        v = ri * ri;
    }
    v = block_sum<double, KNT>(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = v;
    if (!arrive_last(&st->cnt[1], &last)) return;
    const double rr = finish_partials(partial, gridDim.x, sh);
    if (threadIdx.x == 0) {
        st->cnt[1] = 0;
        st->rr = rr;
        st->iters += 1;
        if (!isfinite(rr)) {
            st->done = 1;
            st->status = KS_BREAKDOWN;
        } else if (st->fixed > 0) {
            if (st->iters >= st->fixed) {
                st->done = 1;
                st->status = (rr <= st->rtol2 * st->bb) ? KS_CONVERGED : KS_MAXIT;
            }
        } else if (rr <= st->rtol2 * st->bb) {
            st->done = 1;
            st->status = KS_CONVERGED;
        } else if (st->iters >= st->maxit) {
            st->done = 1;
            st->status = KS_MAXIT;
        }
    }
}

// mode 0: bb = a.b ; mode 1: rho = a.b ; mode 2: beta = a.b / rho, rho = a.b ;
// mode 3: red = a.b (plain dot into st->red)
__global__ __launch_bounds__(KNT) void k_dot(const double *__restrict__ a, const double *__restrict__ b, int n,
                                             double *__restrict__ partial, KState *st, int mode, int cidx) {
    if (mode == 2 && st->done) return;
    __shared__ double sh[KNT / 64];
    __shared__ bool last;
    const int i = blockIdx.x * KNT + threadIdx.x;
    double v = (i < n) ? a[i] * b[i] : 0.0;
    v = block_sum<double, KNT>(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = v;
    if (!arrive_last(&st->cnt[cidx], &last)) return;
    const double t = finish_partials(partial, gridDim.x, sh);
    if (threadIdx.x == 0) {
        st->cnt[cidx] = 0;
        if (mode == 0) st->bb = t;
        else if (mode == 1) st->rho = t;
        else if (mode == 2) {
            if (!isfinite(t) || st->rho == 0.0) {
                st->done = 1;
                st->status = KS_BREAKDOWN;
            } else {
                st->beta = t / st->rho;
                st->rho = t;
            }
        } else {
            st->red = t;
        }
    }
}

// p = z + beta p (init: p = z)
__global__ __launch_bounds__(KNT) void k_cg_update_p(double *__restrict__ p, const double *__restrict__ z, int n,
                                                     const KState *st, int init) {
    if (!init && st->done) return;
    const int i = blockIdx.x * KNT + threadIdx.x;
    if (i >= n) return;
    p[i] = init ? z[i] : z[i] + st->beta * p[i];
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

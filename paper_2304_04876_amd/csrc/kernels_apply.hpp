// Device kernels of the preconditioner apply, eq. (1):
//   one-level part  sum_i R_i^T A_i^{-1} R_i r   (restriction gather, local
//                   solves, deterministic gather-sum), and
//   coarse part     Phi A_0^{-1} Phi^T r        (block GEMV^T, segmented sum,
//                   dense GEMV with the explicit inverse, block GEMV).
#pragma once

#include "kernels_common.hpp"
#include "kernels_setup.hpp"

namespace gdsw {

// ---------------------------------------------------------------------------
// Local ILU(0) solve with Jacobi sweeps (Sec. V-B "Incomplete Local Solver":
// iterative triangular solves, five sweeps by default):
//   y^0 = 0, y^{k+1} = r - N_L y^k;   w^0 = 0, w^{k+1} = D^{-1} y^K - (D^{-1} N_U) w^k.
// One workgroup per subdomain.  Thread t owns rows t, t+NT, ... (R of them);
// its rows' factor entries (KL lower, KU upper slots) stay in registers for
// all sweeps, so the factors are read from HBM once per apply; the two
// iterates live in LDS and alternate.  The inverse pivots (and, for reduced
// precision, the rows' diagonal scale) are staged in LDS with the first
// loads, so that no global load waits in the middle or at the end.  The
// restriction gather (with the optional diagonal scaling of the
// reduced-precision factors) and the write of the local result are fused
// in.  LDS: 3 NT R accumulator values (+ NT R doubles with scaling).
// MS: every right-hand-side slot of the subdomain in one workgroup, one
// after another, with the factor entries loaded once for all of them (the
// slots' sweeps reuse the registers); otherwise the handle has one slot.
template <int NT, int R, int KL, int KU, typename VT, bool MS>
__global__ __launch_bounds__(NT) void k_ilu_jacobi(
    const double *__restrict__ r, const int32_t *__restrict__ ov_idx, const int64_t *__restrict__ ov_ptr,
    const int64_t *__restrict__ ell_off, int64_t ell_rows, const VT *__restrict__ Lv,
    const VT *__restrict__ Uv, const uint32_t *__restrict__ Cp, const VT *__restrict__ dinv,
    const double *__restrict__ dscale, int sweeps, double *__restrict__ zloc, Skip sk) {
    using AT = typename AccOf<VT>::type;
    constexpr int CW = (KL + KU + 1) / 2;   // 32-bit words of packed columns per row
    // FP64 factors are never scaled (dscale is null for them), and their LDS
    // holds no scale slots
    constexpr bool scaled = !std::is_same<VT, double>::value;
    const int i = sk.sub_at(blockIdx.x);
    // (the one-slot form is launched for handles with one slot only: there
    // the slot is the constant 0)
    int slot = 0;
    if constexpr (MS) {
        while (slot < sk.sl.ns && sk.sub(i, slot)) ++slot;
        if (slot == sk.sl.ns) return;
    } else if (sk.sub(i, 0)) {
        return;
    }
    extern __shared__ __align__(16) unsigned char smraw[];
    AT *bufA = reinterpret_cast<AT *>(smraw);
    AT *bufB = bufA + NT * R;
    AT *sdinv = bufB + NT * R;
    double *sscale = reinterpret_cast<double *>(sdinv + NT * R);   // used with dscale only
    const int64_t o = ov_ptr[i];
    const int ni = int(ov_ptr[i + 1] - o);
    const int64_t eo = ell_off[i];
    const int npad = int(ell_off[i + 1] - eo);
    const int tid = threadIdx.x;

    if (ni == 0) return;   // (the whole workgroup)
    __builtin_assume(sweeps >= 2);   // (the launcher takes another kernel for one sweep)
    const int last_r = ni - 1, last_p = npad - 1;
    AT rr[R];
    AT lv[R][KL], uv[R][KU];
    uint32_t cw[R][CW];   // local column of L slot s: half s, of U slot s: half KL + s
    int dof[R];
    // Every load of the thread's rows is issued before any loaded value is
    // used, with no branches between them, in the order the values are
    // needed: the restriction indices, the pivots, the L slots and the
    // columns, the gathered r, and last the U slots, which are only waited
    // for after the L sweeps.  Rows past the subdomain read its last row (in
    // bounds) and are never used.
#pragma unroll
    for (int m = 0; m < R; ++m) dof[m] = ov_idx[o + min(tid + m * NT, last_r)];
    AT dv[R];
#pragma unroll
    for (int m = 0; m < R; ++m) dv[m] = to_acc(ld_once(&dinv[eo + min(tid + m * NT, last_r)]));
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int64_t e = eo + min(tid + m * NT, last_p);
#pragma unroll
        for (int s = 0; s < KL; ++s) lv[m][s] = to_acc(ld_once(&Lv[s * ell_rows + e]));
#pragma unroll
        for (int w = 0; w < CW; ++w) cw[m][w] = ld_once(&Cp[e * CW + w]);
    }
    // the gathered r (scaled for reduced-precision factors)
#pragma unroll
    for (int m = 0; m < R; ++m) {
        double x = r[slot * sk.sl.n + dof[m]];
        if (scaled && dscale) {
            const double sc = dscale[dof[m]];
            x *= sc;
            sscale[tid + m * NT] = sc;
        }
        rr[m] = AT(x);
    }
    // (kept after the loads above by the scheduler barrier)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int64_t e = eo + min(tid + m * NT, last_p);
#pragma unroll
        for (int s = 0; s < KU; ++s) uv[m][s] = to_acc(ld_once(&Uv[s * ell_rows + e]));
    }
    // pivots to LDS for every slot of the thread (rows past the subdomain
    // included: they are never read)
#pragma unroll
    for (int m = 0; m < R; ++m) sdinv[tid + m * NT] = dv[m];
    // The sweeps run over every slot of the thread, rows past the subdomain
    // included (their columns point inside the LDS vectors; no row of the
    // subdomain reads them), so that all LDS reads of a sweep go out before
    // the first product waits.
    AT *cur = bufA, *nxt = bufB;
    for (;;) {   // the right-hand-side slots (one pass unless MS)
    // first L sweep from zero: y^1 = r
#pragma unroll
    for (int m = 0; m < R; ++m) cur[tid + m * NT] = rr[m];
    __syncthreads();
    // rows in groups of SG: the LDS reads of a group are issued together
    constexpr int SG = 4;
    for (int k = 1; k < sweeps; ++k) {
#pragma unroll
        for (int m0 = 0; m0 < R; m0 += SG) {
            AT v[SG][KL];
#pragma unroll
            for (int g = 0; g < SG; ++g)
#pragma unroll
                for (int s = 0; s < KL; ++s)
                    if (m0 + g < R) v[g][s] = cur[(cw[m0 + g][s >> 1] >> (16 * (s & 1))) & 0xffffu];
#pragma unroll
            for (int g = 0; g < SG; ++g)
                if (m0 + g < R) {
                    AT acc = rr[m0 + g];
#pragma unroll
                    for (int s = 0; s < KL; ++s) acc -= lv[m0 + g][s] * v[g][s];
                    nxt[tid + (m0 + g) * NT] = acc;
                }
        }
        __syncthreads();
        AT *t = cur; cur = nxt; nxt = t;
    }
    // c = D^{-1} y^K (kept in rr), first U sweep from zero: w^1 = c (all
    // reads before the writes)
#pragma unroll
    for (int m = 0; m < R; ++m) rr[m] = sdinv[tid + m * NT] * cur[tid + m * NT];
#pragma unroll
    for (int m = 0; m < R; ++m) nxt[tid + m * NT] = rr[m];
    __syncthreads();
    { AT *t = cur; cur = nxt; nxt = t; }
    for (int k = 1; k < sweeps; ++k) {
#pragma unroll
        for (int m0 = 0; m0 < R; m0 += SG) {
            AT v[SG][KU];
#pragma unroll
            for (int g = 0; g < SG; ++g)
#pragma unroll
                for (int s = 0; s < KU; ++s) {
                    const int h = KL + s;
                    if (m0 + g < R) v[g][s] = cur[(cw[m0 + g][h >> 1] >> (16 * (h & 1))) & 0xffffu];
                }
#pragma unroll
            for (int g = 0; g < SG; ++g)
                if (m0 + g < R) {
                    AT acc = rr[m0 + g];
#pragma unroll
                    for (int s = 0; s < KU; ++s) acc -= uv[m0 + g][s] * v[g][s];
                    nxt[tid + (m0 + g) * NT] = acc;
                }
        }
        __syncthreads();
        AT *t = cur; cur = nxt; nxt = t;
    }
    // the result: all LDS reads, then the stores of the subdomain's rows
    double out[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        out[m] = double(cur[tid + m * NT]);
        if (scaled && dscale) out[m] *= sscale[tid + m * NT];
    }
#pragma unroll
    for (int m = 0; m < R; ++m)
        if (tid + m * NT < ni) zloc[slot * sk.sl.zl + o + tid + m * NT] = out[m];
    if constexpr (!MS) {
        break;
    } else {
        // the next slot that runs: its gathered r, after every thread is
        // done with the LDS vectors of this one
        ++slot;
        while (slot < sk.sl.ns && sk.sub(i, slot)) ++slot;
        if (slot == sk.sl.ns) break;
#pragma unroll
        for (int m = 0; m < R; ++m) {
            double x = r[slot * sk.sl.n + dof[m]];
            if (scaled && dscale) x *= sscale[tid + m * NT];
            rr[m] = AT(x);
        }
        __syncthreads();
    }
    }
}

// Same sweeps for any slot counts and subdomain sizes: factors are read from
// global memory on every sweep; r and the iterate pair live in LDS (or in
// global memory when a subdomain does not fit).
template <int NT, typename VT>
__global__ __launch_bounds__(NT) void k_ilu_jacobi_generic(
    const double *__restrict__ r, const int32_t *__restrict__ ov_idx, const int64_t *__restrict__ ov_ptr,
    const int64_t *__restrict__ ell_off, int64_t ell_rows, int KL, int KU, const VT *__restrict__ Lv,
    const uint16_t *__restrict__ Lc, const VT *__restrict__ Uv, const uint16_t *__restrict__ Uc,
    const VT *__restrict__ dinv, const double *__restrict__ dscale, int sweeps,
    double *__restrict__ zloc, int maxrows, void *__restrict__ gbuf, Skip sk) {
    using AT = typename AccOf<VT>::type;
    const int slot = blockIdx.y, i = sk.sub_at(blockIdx.x);
    if (sk.sub(i, slot)) return;
    r += slot * sk.sl.n;
    zloc += slot * sk.sl.zl;
    extern __shared__ __align__(16) unsigned char smraw[];
    const int64_t o = ov_ptr[i];
    const int ni = int(ov_ptr[i + 1] - o);
    // the three vectors live in LDS, or (subdomains too large for it) in a
    // per-subdomain slice of global memory (per slot), which stays in L2
    AT *rb = gbuf ? reinterpret_cast<AT *>(gbuf) + 3 * (slot * sk.sl.zl + o) : reinterpret_cast<AT *>(smraw);
    const int64_t stride = gbuf ? ni : maxrows;
    AT *cur = rb + stride, *nxt = cur + stride;
    const int64_t eo = ell_off[i];
    for (int l = threadIdx.x; l < ni; l += NT) {
        const int d = ov_idx[o + l];
        double x = r[d];
        if (dscale) x *= dscale[d];
        rb[l] = AT(x);
        cur[l] = AT(x);
    }
    __syncthreads();
    // One sweep: nxt = rb - N cur over the K slots of V / C.  Each thread
    // takes its rows RB at a time and the slots SC at a time: the entries and
    // columns of a chunk are loaded together, then the chunk's iterate
    // entries, then the products, each row's in slot order (the order of
    // one row at a time, so the same bits).  Slots past K are neither loaded
    // nor used; rows past the subdomain load its last row and are not
    // written.
    constexpr int RB = 2, SC = 4;   // (measured: 2 x 4 rows x slots ahead of 4 x 4, 4 x 2, 2 x 2 and larger)
    auto sweep = [&](const VT *__restrict__ V, const uint16_t *__restrict__ C, int K) {
        for (int l0 = threadIdx.x; l0 < ni; l0 += NT * RB) {
            AT acc[RB];
#pragma unroll
            for (int b = 0; b < RB; ++b) acc[b] = rb[min(l0 + b * NT, ni - 1)];
            for (int s0 = 0; s0 < K; s0 += SC) {
                AT v[RB][SC];
                int c[RB][SC];
#pragma unroll
                for (int b = 0; b < RB; ++b)
#pragma unroll
                    for (int j = 0; j < SC; ++j) {
                        const int64_t e = int64_t(min(s0 + j, K - 1)) * ell_rows + eo + min(l0 + b * NT, ni - 1);
                        v[b][j] = to_acc(V[e]);
                        c[b][j] = C[e];
                    }
                AT g[RB][SC];
#pragma unroll
                for (int b = 0; b < RB; ++b)
#pragma unroll
                    for (int j = 0; j < SC; ++j) g[b][j] = cur[c[b][j]];
#pragma unroll
                for (int b = 0; b < RB; ++b)
#pragma unroll
                    for (int j = 0; j < SC; ++j)
                        if (s0 + j < K) acc[b] -= v[b][j] * g[b][j];
            }
#pragma unroll
            for (int b = 0; b < RB; ++b)
                if (l0 + b * NT < ni) nxt[l0 + b * NT] = acc[b];
        }
    };
    for (int k = 1; k < sweeps; ++k) {
        sweep(Lv, Lc, KL);
        __syncthreads();
        AT *t = cur; cur = nxt; nxt = t;
    }
    for (int l = threadIdx.x; l < ni; l += NT) {
        rb[l] = to_acc(dinv[eo + l]) * cur[l];
        nxt[l] = rb[l];
    }
    __syncthreads();
    { AT *t = cur; cur = nxt; nxt = t; }
    for (int k = 1; k < sweeps; ++k) {
        sweep(Uv, Uc, KU);
        __syncthreads();
        AT *t = cur; cur = nxt; nxt = t;
    }
    for (int l = threadIdx.x; l < ni; l += NT) {
        double v = double(cur[l]);
        if (dscale) v *= dscale[ov_idx[o + l]];
        zloc[o + l] = v;
    }
}

// ILU(k) factors with more slots per row than the registers hold beside
// the sweeps (ILU(2) and ILU(3) of the 7-point stencil: 11 + 11 and 21 + 21
// slots): the first H slots of each of the thread's R rows stay in registers
// across the sweeps of a triangle (the L slots for the L sweeps, then the U
// slots in the same registers), so that only the slots past them are read
// again on every sweep (two rows and four slots at a time, as in
// k_ilu_jacobi_generic).  Each row's products in slot order: the same bits
// as the streaming sweeps.  Rows t, t + NT, ... of thread t (ni <= NT R and
// the vectors in LDS, checked by the launcher); right-hand-side slot
// blockIdx.y.
template <int NT, int R, int H, typename VT>
__global__ __launch_bounds__(NT) void k_ilu_jacobi_hold(
    const double *__restrict__ r, const int32_t *__restrict__ ov_idx, const int64_t *__restrict__ ov_ptr,
    const int64_t *__restrict__ ell_off, int64_t ell_rows, int KL, int KU, const VT *__restrict__ Lv,
    const uint16_t *__restrict__ Lc, const VT *__restrict__ Uv, const uint16_t *__restrict__ Uc,
    const VT *__restrict__ dinv, const double *__restrict__ dscale, int sweeps,
    double *__restrict__ zloc, int maxrows, Skip sk) {
    using AT = typename AccOf<VT>::type;
    static_assert(H % 2 == 0, "held columns two to a word");
    const int slot = blockIdx.y, i = sk.sub_at(blockIdx.x);
    if (sk.sub(i, slot)) return;
    r += slot * sk.sl.n;
    zloc += slot * sk.sl.zl;
    extern __shared__ __align__(16) unsigned char smraw[];
    const int64_t o = ov_ptr[i];
    const int ni = int(ov_ptr[i + 1] - o);
    if (ni == 0) return;   // (the whole workgroup)
    AT *rb = reinterpret_cast<AT *>(smraw);
    AT *cur = rb + maxrows, *nxt = cur + maxrows;
    const int64_t eo = ell_off[i];
    const int tid = threadIdx.x;
    for (int l = tid; l < ni; l += NT) {
        const int d = ov_idx[o + l];
        double x = r[d];
        if (dscale) x *= dscale[d];
        rb[l] = AT(x);
        cur[l] = AT(x);
    }
    // the held slots of the thread's rows (rows past the subdomain read its
    // last row and are never written)
    AT hv[R][H];
    uint32_t hc[R][H / 2];   // columns of slots j and j + 1 in one word
    auto hold = [&](const VT *__restrict__ V, const uint16_t *__restrict__ C, int K) {
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int64_t e0 = eo + min(tid + m * NT, ni - 1);
#pragma unroll
            for (int j = 0; j < H; j += 2) {
                const int64_t ea = int64_t(min(j, K - 1)) * ell_rows + e0;
                const int64_t eb = int64_t(min(j + 1, K - 1)) * ell_rows + e0;
                hv[m][j] = to_acc(V[ea]);
                hv[m][j + 1] = to_acc(V[eb]);
                hc[m][j / 2] = uint32_t(C[ea]) | (uint32_t(C[eb]) << 16);
            }
        }
    };
    constexpr int SC = 4;
    auto sweep = [&](const VT *__restrict__ V, const uint16_t *__restrict__ C, int K) {
#pragma unroll
        for (int m0 = 0; m0 < R; m0 += 2) {
            AT acc[2];
#pragma unroll
            for (int b = 0; b < 2; ++b)
                if (m0 + b < R) acc[b] = rb[min(tid + (m0 + b) * NT, ni - 1)];
#pragma unroll
            for (int b = 0; b < 2; ++b)
                if (m0 + b < R) {
#pragma unroll
                    for (int j = 0; j < H; ++j)
                        if (j < K) acc[b] -= hv[m0 + b][j] * cur[(hc[m0 + b][j / 2] >> (16 * (j & 1))) & 0xffffu];
                }
            for (int s0 = H; s0 < K; s0 += SC) {
                AT v[2][SC];
                int c[2][SC];
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int j = 0; j < SC; ++j) {
                        const int64_t e = int64_t(min(s0 + j, K - 1)) * ell_rows + eo +
                                          min(tid + min(m0 + b, R - 1) * NT, ni - 1);
                        v[b][j] = to_acc(V[e]);
                        c[b][j] = C[e];
                    }
                AT g[2][SC];
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int j = 0; j < SC; ++j) g[b][j] = cur[c[b][j]];
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    if (m0 + b < R) {
#pragma unroll
                        for (int j = 0; j < SC; ++j)
                            if (s0 + j < K) acc[b] -= v[b][j] * g[b][j];
                    }
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int l = tid + (m0 + b) * NT;
                if (m0 + b < R && l < ni) nxt[l] = acc[b];
            }
        }
    };
    hold(Lv, Lc, KL);
    __syncthreads();
    for (int k = 1; k < sweeps; ++k) {
        sweep(Lv, Lc, KL);
        __syncthreads();
        AT *t = cur; cur = nxt; nxt = t;
    }
    for (int l = tid; l < ni; l += NT) {
        rb[l] = to_acc(dinv[eo + l]) * cur[l];
        nxt[l] = rb[l];
    }
    hold(Uv, Uc, KU);
    __syncthreads();
    { AT *t = cur; cur = nxt; nxt = t; }
    for (int k = 1; k < sweeps; ++k) {
        sweep(Uv, Uc, KU);
        __syncthreads();
        AT *t = cur; cur = nxt; nxt = t;
    }
    for (int l = tid; l < ni; l += NT) {
        double v = double(cur[l]);
        if (dscale) v *= dscale[ov_idx[o + l]];
        zloc[o + l] = v;
    }
}

// The register-resident sweeps for factors with more slots per row (ILU(k)
// with fill: KL = KU = 6 for ILU(1) of the 7-point stencil), whose L and U
// entries do not fit the registers together: the L entries and columns are
// held in registers for the L sweeps, then the same registers take the U
// entries and columns, loaded after the L sweeps, for the U sweeps.  Each
// factor entry is still read once per apply.  One right-hand-side slot;
// the same rows per thread and order of operations as k_ilu_jacobi, so
// the same results as the streaming sweeps bit for bit.  Columns: CW words
// per row, the KL (even) L columns in the first KL/2 words, the U columns
// after them, word w of row e at Cp[w * cps + e] (each phase reads only its
// own words).  The factor rows of a thread are read at fixed strides from
// one base, without clamping: rows past a subdomain's padded rows are the
// next subdomain's, and the arrays carry ILU_PAD_ROWS zeroed rows past the
// last one, so every read is in bounds and every column points inside the
// LDS vectors; those rows' results are never read or stored.  LDS: the two
// iterates (and the scales of reduced-precision factors); the pivots are
// read from memory when the U phase starts.
template <int NT, int R, int KL, int KU, typename VT>
__global__ __launch_bounds__(NT) void k_ilu_jacobi_phased(
    const double *__restrict__ r, const int32_t *__restrict__ ov_idx, const int64_t *__restrict__ ov_ptr,
    const int64_t *__restrict__ ell_off, int64_t ell_rows, const VT *__restrict__ Lv,
    const VT *__restrict__ Uv, const uint32_t *__restrict__ Cp, int64_t cps, const VT *__restrict__ dinv,
    const double *__restrict__ dscale, int sweeps, double *__restrict__ zloc, Skip sk) {
    using AT = typename AccOf<VT>::type;
    static_assert(KL % 2 == 0, "the L columns end on a word boundary");
    constexpr int CW = (KL + KU + 1) / 2, CL = KL / 2, CU = CW - CL;
    constexpr bool scaled = !std::is_same<VT, double>::value;
    constexpr int SG = 2;   // rows whose LDS reads of a sweep are issued together
    const int i = sk.sub_at(blockIdx.x);
    if (sk.sub(i, 0)) return;
    extern __shared__ __align__(16) unsigned char smraw[];
    AT *bufA = reinterpret_cast<AT *>(smraw);
    AT *bufB = bufA + NT * R;
    double *sscale = reinterpret_cast<double *>(bufB + NT * R);   // used with dscale only
    const int64_t o = ov_ptr[i];
    const int ni = int(ov_ptr[i + 1] - o);
    const int64_t eo = ell_off[i];
    const int npad = int(ell_off[i + 1] - eo);
    const int tid = threadIdx.x;
    if (ni == 0) return;   // (the whole workgroup)
    __builtin_assume(sweeps >= 2);
    const int last_r = ni - 1;
    (void)npad;
    AT rr[R];
    AT *cur = bufA, *nxt = bufB;
    {
        int dof[R];
#pragma unroll
        for (int m = 0; m < R; ++m) dof[m] = ov_idx[o + min(tid + m * NT, last_r)];
        AT lv[R][KL];
        uint32_t cw[R][CL];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int64_t e = eo + tid + m * NT;
#pragma unroll
            for (int s = 0; s < KL; ++s) lv[m][s] = to_acc(ld_once(&Lv[s * ell_rows + e]));
#pragma unroll
            for (int w = 0; w < CL; ++w) cw[m][w] = ld_once(&Cp[w * cps + e]);
        }
#pragma unroll
        for (int m = 0; m < R; ++m) {
            double x = r[dof[m]];
            if (scaled && dscale) {
                const double sc = dscale[dof[m]];
                x *= sc;
                sscale[tid + m * NT] = sc;
            }
            rr[m] = AT(x);
        }
        // first L sweep from zero: y^1 = r
#pragma unroll
        for (int m = 0; m < R; ++m) cur[tid + m * NT] = rr[m];
        __syncthreads();
        for (int k = 1; k < sweeps; ++k) {
            // (the packed columns are unpacked anew every sweep: an empty
            // asm statement marks them as changed, so that the compiler
            // does not keep all LDS addresses live across the sweeps)
#pragma unroll
            for (int m = 0; m < R; ++m)
#pragma unroll
                for (int w = 0; w < CL; ++w) asm volatile("" : "+v"(cw[m][w]));
#pragma unroll
            for (int m0 = 0; m0 < R; m0 += SG) {
                AT v[SG][KL];
#pragma unroll
                for (int g = 0; g < SG; ++g)
#pragma unroll
                    for (int s = 0; s < KL; ++s)
                        if (m0 + g < R) v[g][s] = cur[(cw[m0 + g][s >> 1] >> (16 * (s & 1))) & 0xffffu];
#pragma unroll
                for (int g = 0; g < SG; ++g)
                    if (m0 + g < R) {
                        AT acc = rr[m0 + g];
#pragma unroll
                        for (int s = 0; s < KL; ++s) acc -= lv[m0 + g][s] * v[g][s];
                        nxt[tid + (m0 + g) * NT] = acc;
                    }
            }
            __syncthreads();
            AT *t = cur; cur = nxt; nxt = t;
        }
    }
    // c = D^{-1} y^K (kept in rr; the pivots loaded only now, to keep the
    // registers for the L entries), first U sweep from zero: w^1 = c
    {
        AT dv[R];
#pragma unroll
        for (int m = 0; m < R; ++m) dv[m] = to_acc(ld_once(&dinv[eo + min(tid + m * NT, last_r)]));
#pragma unroll
        for (int m = 0; m < R; ++m) rr[m] = dv[m] * cur[tid + m * NT];
    }
#pragma unroll
    for (int m = 0; m < R; ++m) nxt[tid + m * NT] = rr[m];
    {
        // (the row index passes through an empty asm statement after the L
        // sweeps, so that the U loads cannot be hoisted above them and hold
        // registers during the L phase)
        int tu = tid;
        asm volatile("" : "+v"(tu));
        AT uv[R][KU];
        uint32_t cu[R][CU];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int64_t e = eo + tu + m * NT;
#pragma unroll
            for (int s = 0; s < KU; ++s) uv[m][s] = to_acc(ld_once(&Uv[s * ell_rows + e]));
#pragma unroll
            for (int w = 0; w < CU; ++w) cu[m][w] = ld_once(&Cp[(CL + w) * cps + e]);
        }
        __syncthreads();
        { AT *t = cur; cur = nxt; nxt = t; }
        for (int k = 1; k < sweeps; ++k) {
#pragma unroll
            for (int m = 0; m < R; ++m)
#pragma unroll
                for (int w = 0; w < CU; ++w) asm volatile("" : "+v"(cu[m][w]));
#pragma unroll
            for (int m0 = 0; m0 < R; m0 += SG) {
                AT v[SG][KU];
#pragma unroll
                for (int g = 0; g < SG; ++g)
#pragma unroll
                    for (int s = 0; s < KU; ++s)
                        if (m0 + g < R) v[g][s] = cur[(cu[m0 + g][s >> 1] >> (16 * (s & 1))) & 0xffffu];
#pragma unroll
                for (int g = 0; g < SG; ++g)
                    if (m0 + g < R) {
                        AT acc = rr[m0 + g];
#pragma unroll
                        for (int s = 0; s < KU; ++s) acc -= uv[m0 + g][s] * v[g][s];
                        nxt[tid + (m0 + g) * NT] = acc;
                    }
            }
            __syncthreads();
            AT *t = cur; cur = nxt; nxt = t;
        }
    }
    double out[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        out[m] = double(cur[tid + m * NT]);
        if (scaled && dscale) out[m] *= sscale[tid + m * NT];
    }
#pragma unroll
    for (int m = 0; m < R; ++m)
        if (tid + m * NT < ni) zloc[o + tid + m * NT] = out[m];
}

// ---------------------------------------------------------------------------
// Exact local solve A_i^{-1} r_i with the banded Cholesky factor, one
// workgroup per subdomain, vector in LDS, gather and scatter fused.
template <int NT, typename VT, bool INV, bool AHEAD>
__device__ __forceinline__ void band_apply_one(int i, const double *__restrict__ r, const int32_t *__restrict__ ov_idx,
                                               const int64_t *__restrict__ ov_ptr, const VT *__restrict__ band,
                                               const int64_t *__restrict__ band_off, const int32_t *__restrict__ bw,
                                               const double *__restrict__ dscale, double *__restrict__ zloc,
                                               int maxrows) {
    using AT = typename AccOf<VT>::type;
    extern __shared__ __align__(16) unsigned char smraw[];
    AT *y = reinterpret_cast<AT *>(smraw);
    AT *sT = y + maxrows;
    const int64_t o = ov_ptr[i];
    const int ni = int(ov_ptr[i + 1] - o);
    // gathers and stores in batches of GB rows per thread, every load of a
    // batch issued before the first use (rows past the end re-read the last)
    constexpr int GB = 4;
    for (int l0 = threadIdx.x; l0 < ni; l0 += GB * NT) {
        int d[GB];
#pragma unroll
        for (int b = 0; b < GB; ++b) d[b] = ov_idx[o + min(l0 + b * NT, ni - 1)];
        double x[GB];
#pragma unroll
        for (int b = 0; b < GB; ++b) x[b] = r[d[b]];
        if (dscale) {
            double sc[GB];
#pragma unroll
            for (int b = 0; b < GB; ++b) sc[b] = dscale[d[b]];
#pragma unroll
            for (int b = 0; b < GB; ++b) x[b] *= sc[b];
        }
#pragma unroll
        for (int b = 0; b < GB; ++b)
            if (l0 + b * NT < ni) y[l0 + b * NT] = AT(x[b]);
    }
    __syncthreads();
    band_llt_solve<VT, AT, NT, INV, AHEAD>(band + band_off[i], ni, bw[i], y, sT);
    for (int l0 = threadIdx.x; l0 < ni; l0 += GB * NT) {
        double v[GB];
#pragma unroll
        for (int b = 0; b < GB; ++b) v[b] = double(y[min(l0 + b * NT, ni - 1)]);
        if (dscale) {
            int d[GB];
#pragma unroll
            for (int b = 0; b < GB; ++b) d[b] = ov_idx[o + min(l0 + b * NT, ni - 1)];
            double sc[GB];
#pragma unroll
            for (int b = 0; b < GB; ++b) sc[b] = dscale[d[b]];
#pragma unroll
            for (int b = 0; b < GB; ++b) v[b] *= sc[b];
        }
#pragma unroll
        for (int b = 0; b < GB; ++b)
            if (l0 + b * NT < ni) zloc[o + l0 + b * NT] = v[b];
    }
}

// (compiled for up to 1024 threads whatever NT is: that register budget
// keeps the unrolled triangle solve from spilling)
template <int NT, typename VT, bool INV>
__global__ __launch_bounds__(1024) void k_band_apply(
    const double *__restrict__ r, const int32_t *__restrict__ ov_idx, const int64_t *__restrict__ ov_ptr,
    const VT *__restrict__ band, const int64_t *__restrict__ band_off, const int32_t *__restrict__ bw,
    const double *__restrict__ dscale, double *__restrict__ zloc, int maxrows, Skip sk) {
    const int slot = blockIdx.y, i = sk.sub_at(blockIdx.x);
    // (subdomains without a band take the supernodal solve)
    if (sk.sub(i, slot) || band_inverted(bw[i]) != INV || band_off[i + 1] == band_off[i]) return;
    band_apply_one<NT, VT, INV, true>(i, r + slot * sk.sl.n, ov_idx, ov_ptr, band, band_off, bw, dscale,
                                      zloc + slot * sk.sl.zl, maxrows);
}

// The same as a persistent loop: gridDim.x workgroups per slot take the
// launch order's subdomains from a work counter (queue[slot], zeroed by the
// launcher before the launch) until all `nitems` are taken; with the order
// by decreasing size this is a largest-first list scheduled dynamically.
template <int NT, typename VT, bool INV>
__global__ __launch_bounds__(1024) void k_band_apply_pers(
    const double *__restrict__ r, const int32_t *__restrict__ ov_idx, const int64_t *__restrict__ ov_ptr,
    const VT *__restrict__ band, const int64_t *__restrict__ band_off, const int32_t *__restrict__ bw,
    const double *__restrict__ dscale, double *__restrict__ zloc, int maxrows, Skip sk, int *__restrict__ queue,
    int nitems) {
    __shared__ int s_t;
    const int slot = blockIdx.y;
    for (;;) {
        if (threadIdx.x == 0) s_t = atomicAdd(&queue[slot], 1);
        __syncthreads();
        const int t = s_t;
        __syncthreads();   // (every thread has read the ticket before the next is drawn)
        if (t >= nitems) break;   // (the whole workgroup)
        const int i = sk.sub_at(t);
        if (!sk.sub(i, slot) && band_inverted(bw[i]) == INV && band_off[i + 1] != band_off[i])
            band_apply_one<NT, VT, INV, false>(i, r + slot * sk.sl.n, ov_idx, ov_ptr, band, band_off, bw, dscale,
                                               zloc + slot * sk.sl.zl, maxrows);
        __syncthreads();   // (the LDS vector is free for the next subdomain)
    }
}

// ---------------------------------------------------------------------------
// Coarse restriction Phi^T r.  Each block B_g (rows_g x k_g, column-major)
// contributes partial sums of its columns; a column's partials are added in
// a fixed order by k_coarse_reduce.  Blocks of many rows (subdomain
// interiors) are cut into tiles of at most 1024 rows, one 256-thread
// workgroup per tile (4 rows per thread, every load of a pass issued before
// the sums); small blocks (interface components) take a wavefront each.
// Up to 8 columns per pass; a tile's columns are cut into chunks of RT_CK,
// one workgroup per chunk (each partial is still formed by one workgroup,
// in the same order).
constexpr int RT_NT = 256, RT_RPT = 4, RT_ROWS = RT_NT * RT_RPT, RT_KB = 8, RT_CK = 32;

template <typename PT>
__device__ __forceinline__ void restrict_tile(const double *__restrict__ r, const int64_t *__restrict__ row_ptr,
                                              const int32_t *__restrict__ rows, const int64_t *__restrict__ col_ptr,
                                              const int64_t *__restrict__ val_off, const PT *__restrict__ phi, int g,
                                              int l0, int l1, int64_t po, int sbeg, int send,
                                              double *__restrict__ partial, double (*sh)[RT_NT / 64]) {
    constexpr int KB = RT_KB, NW = RT_NT / 64;
    const int64_t r0 = row_ptr[g];
    const int nr = int(row_ptr[g + 1] - r0);
    const int k = min(int(col_ptr[g + 1] - col_ptr[g]), send);
    const PT *Bg = phi + val_off[g];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // rows past the tile and columns past the block read the tile's last row
    // and the block's last column (in bounds, no branch between the loads);
    // x is zero there, so they add nothing to the columns that are written
    if (l1 <= l0) {   // an empty tile (the whole workgroup): zero partials
        for (int s = sbeg + tid; s < k; s += RT_NT) partial[po + s] = 0.0;
        return;
    }
    int ri[RT_RPT];
#pragma unroll
    for (int j = 0; j < RT_RPT; ++j) ri[j] = rows[r0 + min(l0 + tid + j * RT_NT, l1 - 1)];
    double x[RT_RPT];
#pragma unroll
    for (int j = 0; j < RT_RPT; ++j) {
        const double v = r[ri[j]];
        x[j] = l0 + tid + j * RT_NT < l1 ? v : 0.0;
    }
    for (int s0 = sbeg; s0 < k; s0 += KB) {
        double bv[KB][RT_RPT];
#pragma unroll
        for (int s = 0; s < KB; ++s)
#pragma unroll
            for (int j = 0; j < RT_RPT; ++j) {
                const int l = min(l0 + tid + j * RT_NT, l1 - 1);
                bv[s][j] = double(to_acc(Bg[int64_t(min(s0 + s, k - 1)) * nr + l]));
            }
        double acc[KB];
#pragma unroll
        for (int s = 0; s < KB; ++s) {
            acc[s] = 0.0;
#pragma unroll
            for (int j = 0; j < RT_RPT; ++j) acc[s] += bv[s][j] * x[j];
            acc[s] = wave_sum(acc[s]);
        }
        if (lane == 0)
#pragma unroll
            for (int s = 0; s < KB; ++s) sh[s][wv] = acc[s];
        __syncthreads();
        if (tid < KB && s0 + tid < k) {
            double v = sh[tid][0];
#pragma unroll
            for (int w = 1; w < NW; ++w) v += sh[tid][w];
            partial[po + s0 + tid] = v;
        }
        __syncthreads();
    }
}

template <typename PT>
__device__ __forceinline__ void restrict_wave(const double *__restrict__ r, const int64_t *__restrict__ row_ptr,
                                              const int32_t *__restrict__ rows, const int64_t *__restrict__ col_ptr,
                                              const int64_t *__restrict__ val_off, const PT *__restrict__ phi, int g,
                                              int64_t po, double *__restrict__ partial) {
    const int lane = threadIdx.x & 63;
    const int64_t r0 = row_ptr[g];
    const int nr = int(row_ptr[g + 1] - r0);
    const int k = int(col_ptr[g + 1] - col_ptr[g]);
    const PT *Bg = phi + val_off[g];
    constexpr int KB = RT_KB;
    for (int s0 = 0; s0 < k; s0 += KB) {
        double acc[KB];
#pragma unroll
        for (int s = 0; s < KB; ++s) acc[s] = 0.0;
        // rows in batches of WB per lane, every load of a batch issued before
        // the products (rows past the block re-read its last row, with x = 0);
        // each column adds its rows in the order l = lane, lane + 64, ...
        constexpr int WB = 4;
        for (int l0 = lane; l0 < nr; l0 += WB * 64) {
            int ri[WB];
#pragma unroll
            for (int j = 0; j < WB; ++j) ri[j] = rows[r0 + min(l0 + j * 64, nr - 1)];
            double bv[WB][KB];
#pragma unroll
            for (int j = 0; j < WB; ++j)
#pragma unroll
                for (int s = 0; s < KB; ++s)
                    bv[j][s] = s0 + s < k ? double(to_acc(Bg[int64_t(s0 + s) * nr + min(l0 + j * 64, nr - 1)])) : 0.0;
            double x[WB];
#pragma unroll
            for (int j = 0; j < WB; ++j) {
                const double v = r[ri[j]];
                x[j] = l0 + j * 64 < nr ? v : 0.0;
            }
#pragma unroll
            for (int j = 0; j < WB; ++j)
#pragma unroll
                for (int s = 0; s < KB; ++s)
                    if (s0 + s < k) acc[s] += bv[j][s] * x[j];
        }
#pragma unroll
        for (int s = 0; s < KB; ++s) {
            const double t = wave_sum(acc[s]);
            if (lane == 0 && s0 + s < k) partial[po + s0 + s] = t;
        }
    }
}

// One launch for both kinds: workgroups [0, nwork) take the column chunks
// of the tiles of the big blocks (work item b: tile wk_tile[b], columns from
// wk_s0[b]), the rest four small blocks each (blocks g_small, g_small+1, ...
// below nb), so the short component blocks run beside the tiles.
template <typename PT>
__global__ __launch_bounds__(RT_NT) void k_coarse_restrict(
    const double *__restrict__ r, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ rows,
    const int64_t *__restrict__ col_ptr, const int64_t *__restrict__ val_off, const PT *__restrict__ phi,
    const int32_t *__restrict__ tile_blk, const int32_t *__restrict__ tile_l0, const int32_t *__restrict__ tile_l1,
    const int64_t *__restrict__ tile_poff, const int32_t *__restrict__ wk_tile, const int32_t *__restrict__ wk_s0,
    const int64_t *__restrict__ poff, double *__restrict__ partial, int nwork, int g_small, int nb, Skip sk) {
    __shared__ double sh[RT_KB][RT_NT / 64];
    const int b = blockIdx.x, slot = blockIdx.y;
    r += slot * sk.sl.n;
    partial += slot * sk.sl.part;
    if (b < nwork) {
        const int t = wk_tile[b], g = tile_blk[t];
        if (sk.blk(g, slot)) return;
        const int s0 = wk_s0[b];
        restrict_tile<PT>(r, row_ptr, rows, col_ptr, val_off, phi, g, tile_l0[t], tile_l1[t], tile_poff[t], s0,
                          s0 + RT_CK, partial, sh);
    } else {
        const int g = g_small + (b - nwork) * (RT_NT / 64) + int(threadIdx.x >> 6);
        if (g >= nb || sk.blk(g, slot)) return;
        restrict_wave<PT>(r, row_ptr, rows, col_ptr, val_off, phi, g, poff[g], partial);
    }
}

// r0[c] = sum of the partials of coarse column c (ascending block order)
// One wavefront per column: lane j adds partials j, j + 64, ... of the
// column's list, then the wavefront sum (a fixed order that depends only on
// the column's list).
__global__ __launch_bounds__(256) void k_coarse_reduce(const int64_t *__restrict__ red_ptr,
                                                       const int32_t *__restrict__ red_idx,
                                                       const double *__restrict__ partial, double *__restrict__ r0,
                                                       int n0, Skip sk) {
    const int c = blockIdx.x * 4 + int(threadIdx.x >> 6), lane = threadIdx.x & 63, slot = blockIdx.y;
    if (c >= n0 || sk.col(c, slot)) return;   // (the whole wavefront)
    partial += slot * sk.sl.part;
    r0 += slot * sk.sl.n0;
    const int64_t q1 = red_ptr[c + 1];
    double acc = 0.0;
    for (int64_t q = red_ptr[c] + lane; q < q1; q += 64) acc += partial[red_idx[q]];
    acc = wave_sum(acc);
    if (lane == 0) r0[c] = acc;
}

// z0 = A_0^{-1} r0 with A_0^{-1} block diagonal over the problems of the
// handle (row-major dense blocks): one wavefront per row.  Each result is
// also written to zg at every position where its column appears in the
// column lists of the coarse basis blocks (cpos_ptr/cpos), so that the
// prolongation reads z0 in block-column order without the index gather.
__global__ __launch_bounds__(256) void k_block_gemv(const double *__restrict__ Ainv, const int64_t *__restrict__ a0_off,
                                                    const int32_t *__restrict__ prob_c0,
                                                    const int32_t *__restrict__ cprob, const double *__restrict__ x,
                                                    double *__restrict__ y, const int64_t *__restrict__ cpos_ptr,
                                                    const int32_t *__restrict__ cpos, double *__restrict__ zg, int n0,
                                                    Skip sk) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, slot = blockIdx.y;
    if (row >= n0 || sk.col(row, slot)) return;
    x += slot * sk.sl.n0;
    y += slot * sk.sl.n0;
    zg += slot * sk.sl.cols;
    const int k = cprob[row];
    const int c0 = prob_c0[k], nk = prob_c0[k + 1] - c0;
    const double *a = Ainv + a0_off[k] + int64_t(row - c0) * nk;
    const double *xk = x + c0;
    constexpr int U = 8;
    double acc = 0.0;
    for (int c0 = lane; c0 < nk; c0 += U * 64) {
        double av[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = c0 + u * 64;
            av[u] = c < nk ? ld_once(&a[c]) : 0.0;
            xv[u] = c < nk ? xk[c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c0 + u * 64 < nk) acc += av[u] * xv[u];
    }
    acc = wave_sum(acc);
    if (lane == 0) y[row] = acc;
    for (int64_t p = cpos_ptr[row] + lane; p < cpos_ptr[row + 1]; p += 64) zg[cpos[p]] = acc;
}

// Same with one workgroup (4 wavefronts) per row, for blocks of large order:
// GW_R consecutive rows per workgroup, which read each entry of r0 once for
// all of them when they belong to one problem.  Each row's products are
// added per thread in column order and then summed over the workgroup as
// for a single row, so the rows do not change each other's bits.
constexpr int GW_R = 4;
__global__ __launch_bounds__(256) void k_block_gemv_wg(const double *__restrict__ Ainv, const int64_t *__restrict__ a0_off,
                                                       const int32_t *__restrict__ prob_c0,
                                                       const int32_t *__restrict__ cprob, const double *__restrict__ x,
                                                       double *__restrict__ y, const int64_t *__restrict__ cpos_ptr,
                                                       const int32_t *__restrict__ cpos, double *__restrict__ zg,
                                                       int n0, Skip sk) {
    __shared__ double sh[GW_R][4];
    const int r0 = blockIdx.x * GW_R, slot = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int row[GW_R];
    bool act[GW_R];
    bool any = false;
#pragma unroll
    for (int j = 0; j < GW_R; ++j) {
        row[j] = min(r0 + j, n0 - 1);
        act[j] = r0 + j < n0 && !sk.col(row[j], slot);
        any |= act[j];
    }
    if (!any) return;   // (the whole workgroup)
    x += slot * sk.sl.n0;
    y += slot * sk.sl.n0;
    zg += slot * sk.sl.cols;
    const int k0 = cprob[row[0]];
    bool same = true;
#pragma unroll
    for (int j = 1; j < GW_R; ++j) same &= cprob[row[j]] == k0;
    constexpr int U = 12;
    double acc[GW_R];
#pragma unroll
    for (int j = 0; j < GW_R; ++j) acc[j] = 0.0;
    if (same) {
        const int c0 = prob_c0[k0], nk = prob_c0[k0 + 1] - c0;
        const double *xk = x + c0;
        const double *a0 = Ainv + a0_off[k0];
        for (int cc = tid; cc < nk; cc += U * 256) {
            double xv[U], av[GW_R][U];
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = cc + u * 256 < nk ? xk[cc + u * 256] : 0.0;
#pragma unroll
            for (int j = 0; j < GW_R; ++j)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    av[j][u] = cc + u * 256 < nk ? ld_once(&a0[int64_t(row[j] - c0) * nk + cc + u * 256]) : 0.0;
#pragma unroll
            for (int j = 0; j < GW_R; ++j)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (cc + u * 256 < nk) acc[j] += av[j][u] * xv[u];
        }
    } else {   // rows of different problems (problem boundaries of a batch)
#pragma unroll
        for (int j = 0; j < GW_R; ++j) {
            const int k = cprob[row[j]];
            const int c0 = prob_c0[k], nk = prob_c0[k + 1] - c0;
            const double *a = Ainv + a0_off[k] + int64_t(row[j] - c0) * nk;
            for (int c = tid; c < nk; c += 256) acc[j] += ld_once(&a[c]) * x[c0 + c];
        }
    }
    // the workgroup sums, as block_sum for each row
#pragma unroll
    for (int j = 0; j < GW_R; ++j) {
        const double v = wave_sum(acc[j]);
        if (lane == 0) sh[j][wv] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < GW_R; ++j) {
        double t = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) t += sh[j][w];
        if (!act[j]) continue;
        if (tid == 0) y[row[j]] = t;
        for (int64_t p = cpos_ptr[row[j]] + tid; p < cpos_ptr[row[j] + 1]; p += 256) zg[cpos[p]] = t;
    }
}

// Coarse part of the prolongation by blocks, for coarse bases with many
// columns per block: zc[rows of B_g] = B_g z0(cols_g), z0(cols_g) read from
// the gathered copy zg.  A tile of a big
// block per workgroup (RT_RPT rows per thread, the block's z0 entries staged
// in LDS, columns in passes of RT_KB with every load of a pass issued first)
// and a wavefront per small block.  Each row adds its products in column
// order from zero, the order of the per-dof form below, so both forms give
// the same bits.
template <typename PT>
__global__ __launch_bounds__(RT_NT) void k_coarse_prolong(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ rows, const int64_t *__restrict__ col_ptr,
    const int64_t *__restrict__ val_off, const PT *__restrict__ phi, const int32_t *__restrict__ tile_blk,
    const int32_t *__restrict__ tile_l0, const int32_t *__restrict__ tile_l1, const double *__restrict__ zg,
    double *__restrict__ zc, int ntiles, int g_small, int nb, Skip sk) {
    extern __shared__ double sz[];   // z0 entries of the tile's block (max columns of a big block)
    const int b = blockIdx.x, tid = threadIdx.x, slot = blockIdx.y;
    zg += slot * sk.sl.cols;
    zc += slot * sk.sl.n;
    if (b < ntiles * RT_RPT) {
        // quarter q of tile t: rows l0 + q * RT_NT + tid, one per thread
        const int t = b / RT_RPT, q = b % RT_RPT;
        const int g = tile_blk[t];
        if (sk.blk(g, slot)) return;
        const int64_t r0 = row_ptr[g];
        const int nr = int(row_ptr[g + 1] - r0);
        const int64_t c0 = col_ptr[g];
        const int k = int(col_ptr[g + 1] - c0);
        const int l = tile_l0[t] + q * RT_NT + tid, l1 = tile_l1[t];
        if (tile_l0[t] + q * RT_NT >= l1) return;   // empty quarter (uniform over the workgroup)
        const PT *Bg = phi + val_off[g];
        for (int c = tid; c < k; c += RT_NT) sz[c] = zg[c0 + c];
        __syncthreads();
        double acc = 0.0;
        constexpr int KB = 16;
        for (int s0 = 0; s0 < k; s0 += KB) {
            double bv[KB];
#pragma unroll
            for (int s = 0; s < KB; ++s)
                bv[s] = (s0 + s < k && l < l1) ? double(to_acc(Bg[int64_t(s0 + s) * nr + l])) : 0.0;
#pragma unroll
            for (int s = 0; s < KB; ++s)
                if (s0 + s < k) acc += bv[s] * sz[s0 + s];
        }
        if (l < l1) zc[rows[r0 + l]] = acc;
    } else {
        const int g = g_small + (b - ntiles * RT_RPT) * (RT_NT / 64) + (tid >> 6);
        if (g >= nb || sk.blk(g, slot)) return;
        const int64_t r0 = row_ptr[g];
        const int nr = int(row_ptr[g + 1] - r0);
        const int64_t c0 = col_ptr[g];
        const int k = int(col_ptr[g + 1] - c0);
        const PT *Bg = phi + val_off[g];
        for (int l = tid & 63; l < nr; l += 64) {
            double acc = 0.0;
            for (int s = 0; s < k; ++s) acc += double(to_acc(Bg[int64_t(s) * nr + l])) * zg[c0 + s];
            zc[rows[r0 + l]] = acc;
        }
    }
}

// z[d] = sum over the local rows holding d (ascending subdomain) of zloc
//        + Phi(d, :) z0       (W: bit 0 one-level part, bit 1 coarse part;
//        z0 read in block-column order from zg)
// BLK: the coarse part was formed by blocks (k_coarse_prolong) into zc.
// The parts and the form are template arguments, so that the loads below
// form straight-line code the compiler can issue in three waves, each before
// anything waits for it: (1) where the local rows of d start and end, the
// block and row of d in the coarse basis; (2) the first local row and the
// block's shape; (3) the first local result, the first chunk of d's row of
// the basis and of z0.
template <typename PT, int W, bool BLK>
__device__ __forceinline__ double prolong_one(int64_t d, const int32_t *__restrict__ t_ptr,
                                              const int32_t *__restrict__ t_pos, const double *__restrict__ zloc,
                                              const int32_t *__restrict__ dof_blk, const int32_t *__restrict__ dof_lr,
                                              const int64_t *__restrict__ row_ptr, const int64_t *__restrict__ col_ptr,
                                              const int64_t *__restrict__ val_off, const PT *__restrict__ phi,
                                              const double *__restrict__ zg, const double *__restrict__ zc) {
    constexpr bool one = (W & 1) != 0, two = (W & 2) != 0, by_dof = two && !BLK;
    constexpr int U = 8;   // columns per chunk
    int p0 = 0, p1 = 0, g = -1, lr = 0;
    if constexpr (one) {
        p0 = t_ptr[d];
        p1 = t_ptr[d + 1];
    }
    if constexpr (two) g = dof_blk[d];
    if constexpr (by_dof) lr = dof_lr[d];
    // (every dof lies in at least one overlapping subdomain, and a coarse
    // part means at least one block: the loads stay in bounds; values read
    // for a dof outside the coarse basis, g < 0, are not used)
    const int gg = max(g, 0);
    int64_t rp0 = 0, rp1 = 0, c0 = 0, c1 = 0, vo = 0;
    if constexpr (by_dof) {
        rp0 = row_ptr[gg];
        rp1 = row_ptr[gg + 1];
        c0 = col_ptr[gg];
        c1 = col_ptr[gg + 1];
        vo = val_off[gg];
    }
    double z_first = 0.0, zc_d = 0.0;
    if constexpr (one) z_first = zloc[t_pos[p0]];
    if constexpr (two && BLK) zc_d = zc[d];
    const int64_t nr = rp1 - rp0;
    const int k = g >= 0 ? int(c1 - c0) : 0;
    const PT *Bg = phi + vo + lr;
    double bv[U], zv[U];
    if constexpr (by_dof) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            bv[u] = u < k ? double(to_acc(Bg[u * nr])) : 0.0;
            zv[u] = u < k ? zg[c0 + u] : 0.0;
        }
    }
    // sums: the local results in ascending subdomain, then the coarse part
    // (its products in column order)
    double acc = 0.0;
    if constexpr (one) {
        acc += z_first;
        for (int p = p0 + 1; p < p1; ++p) acc += zloc[t_pos[p]];
    }
    if constexpr (two && BLK) {
        if (g >= 0) acc += zc_d;
    }
    if constexpr (by_dof) {
        if (g >= 0) {
            double s = 0.0;
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (u < k) s += bv[u] * zv[u];
            for (int q = U; q < k; q += U) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    bv[u] = q + u < k ? double(to_acc(Bg[(q + u) * nr])) : 0.0;
                    zv[u] = q + u < k ? zg[c0 + q + u] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (q + u < k) s += bv[u] * zv[u];
            }
            acc += s;
        }
    }
    return acc;
}

template <typename PT, int W, bool BLK>
__global__ void k_prolong(const int32_t *__restrict__ t_ptr, const int32_t *__restrict__ t_pos,
                          const double *__restrict__ zloc, const int32_t *__restrict__ dof_blk,
                          const int32_t *__restrict__ dof_lr, const int64_t *__restrict__ row_ptr,
                          const int64_t *__restrict__ col_ptr, const int64_t *__restrict__ val_off,
                          const PT *__restrict__ phi, const double *__restrict__ zg, const double *__restrict__ zc,
                          double *__restrict__ z, int64_t n, Skip sk) {
    const int64_t d = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int slot = blockIdx.y;
    if (d >= n || sk.dof(d, slot)) return;
    z[slot * sk.sl.n + d] = prolong_one<PT, W, BLK>(d, t_ptr, t_pos, zloc + slot * sk.sl.zl, dof_blk, dof_lr, row_ptr,
                                                    col_ptr, val_off, phi, zg + slot * sk.sl.cols,
                                                    zc + slot * sk.sl.n);
}

// The same over the row blocks of the Krylov iteration (256 threads, rows
// [row0[b], row1[b]) of one problem in one slot: rows of slot k are
// k n + d), also writing the block's partial of r . z for the next CG step.
template <typename PT, int W, bool BLK>
__global__ __launch_bounds__(256) void k_prolong_dot(
    const int32_t *__restrict__ t_ptr, const int32_t *__restrict__ t_pos, const double *__restrict__ zloc,
    const int32_t *__restrict__ dof_blk, const int32_t *__restrict__ dof_lr, const int64_t *__restrict__ row_ptr,
    const int64_t *__restrict__ col_ptr, const int64_t *__restrict__ val_off, const PT *__restrict__ phi,
    const double *__restrict__ zg, const double *__restrict__ zc, double *__restrict__ z, Skip sk,
    const int32_t *__restrict__ kb_row0, const int32_t *__restrict__ kb_row1, const double *__restrict__ rvec,
    double *__restrict__ partial) {
    __shared__ double sh[4];
    const int blk = blockIdx.x;
    const int row0 = kb_row0[blk], row1 = kb_row1[blk];
    const int slot = sk.sl.ns > 1 ? int(row0 / sk.sl.n) : 0;
    const int64_t base = slot * sk.sl.n;
    if (sk.dof(row0 - base, slot)) return;
    zloc += slot * sk.sl.zl;
    zg += slot * sk.sl.cols;
    zc += base;
    double dot = 0.0;
    for (int v = row0 + threadIdx.x; v < row1; v += 256) {
        const int64_t d = v - base;
        const double val =
            prolong_one<PT, W, BLK>(d, t_ptr, t_pos, zloc, dof_blk, dof_lr, row_ptr, col_ptr, val_off, phi, zg, zc);
        z[v] = val;
        dot += rvec[v] * val;
    }
    dot = block_sum<double, 256>(dot, sh);
    if (threadIdx.x == 0) partial[blk] = dot;
}

}  // namespace gdsw

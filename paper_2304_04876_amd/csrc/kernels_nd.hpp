// Device kernels of the nested-dissection supernodal exact local solver
// (Sec. V-B, sparse direct factorization; the symbolic structure is built on
// the host by nd.cpp).  One workgroup per subdomain throughout.
//
// Panels (factorization): supernode J holds L's columns first_J .. first_J +
// ncol_J - 1 on its own rows and then on its struct rows, column-major with
// leading dimension nrow_J (value index voff_J + c nrow_J + row).  After the
// factorization each diagonal block is replaced by its inverse (lower
// triangular), so that every diagonal step of the solves is one product.
// Solve layout (k_nd_split): the same values of J at the same offset voff_J,
// first the inverted diagonal block (ncol_J x ncol_J, column-major) and
// then the struct part (ns_J x ncol_J, column-major, ns_J = nrow_J -
// ncol_J), so that the solve's diagonal passes and struct passes read
// disjoint cache lines.
#pragma once

#include "kernels_common.hpp"

namespace gdsw {

// Left-looking supernodal Cholesky of the panels of every subdomain (FP64,
// in place; the panels hold A_i's lower entries on entry).  Supernodes in
// children-first order: J first takes the update of every earlier K whose
// struct meets J's columns (up lists: struct(K) from index s0 on lies at
// J's panel rows rel[...], its first n1 rows among J's columns), then its
// own dense Cholesky, column by column.  status[i] = 1 + new local row of a
// non-positive pivot.
template <int NT>
__global__ __launch_bounds__(NT) void k_nd_factor(
    double *__restrict__ P, const int64_t *__restrict__ sn_ptr, const int32_t *__restrict__ first,
    const int32_t *__restrict__ ncol, const int32_t *__restrict__ nrow, const int64_t *__restrict__ voff,
    const int64_t *__restrict__ st_ptr, const int64_t *__restrict__ up_ptr, const int32_t *__restrict__ up_k,
    const int32_t *__restrict__ up_s0, const int32_t *__restrict__ up_n1, const int64_t *__restrict__ up_rel,
    const int32_t *__restrict__ rel, int *__restrict__ status) {
    __shared__ double s_piv;
    const int i = blockIdx.x, tid = threadIdx.x;
    for (int64_t J = sn_ptr[i]; J < sn_ptr[i + 1]; ++J) {
        const int nJ = ncol[J], ldJ = nrow[J];
        double *PJ = P + voff[J];
        for (int64_t u = up_ptr[J]; u < up_ptr[J + 1]; ++u) {
            const int K = up_k[u], s0 = up_s0[u], n1 = up_n1[u];
            const int nK = ncol[K], ldK = nrow[K];
            const double *PK = P + voff[K];
            const int n2 = int(st_ptr[K + 1] - st_ptr[K]) - s0;
            const int32_t *rl = rel + up_rel[u];
            const int base = nK + s0;   // panel row of struct(K)[s0] in K's panel
            // (a, b): consecutive threads take consecutive rows a
            for (int e = tid; e < n2 * n1; e += NT) {
                const int a = e % n2, b = e / n2;
                const int pa = rl[a], pb = rl[b];
                if (pa < pb) continue;
                double acc = 0.0;
                for (int k = 0; k < nK; ++k) acc += PK[int64_t(k) * ldK + base + a] * PK[int64_t(k) * ldK + base + b];
                PJ[int64_t(pb) * ldJ + pa] -= acc;
            }
            __syncthreads();
        }
        for (int j = 0; j < nJ; ++j) {
            if (tid == 0) {
                double d = PJ[int64_t(j) * ldJ + j];
                if (!(d > 0.0)) {
                    atomicCAS(status + i, 0, 1 + first[J] + j);
                    d = 1.0;
                }
                s_piv = sqrt(d);
                PJ[int64_t(j) * ldJ + j] = s_piv;
            }
            __syncthreads();
            const double inv = 1.0 / s_piv;
            for (int r = j + 1 + tid; r < ldJ; r += NT) PJ[int64_t(j) * ldJ + r] *= inv;
            __syncthreads();
            // rank-one update of columns j+1 .. nJ-1 on their rows r >= c
            const int nt = nJ - j - 1, nr = ldJ - j - 1;
            for (int e = tid; e < nt * nr; e += NT) {
                const int c = j + 1 + e / nr, r = j + 1 + e % nr;
                if (r >= c) PJ[int64_t(c) * ldJ + r] -= PJ[int64_t(j) * ldJ + r] * PJ[int64_t(j) * ldJ + c];
            }
            __syncthreads();
        }
    }
}

// Each diagonal block L_JJ replaced by its inverse, in place, from the last
// column to the first: with the trailing block already inverted (M^{-1}),
// column j below the diagonal becomes -M^{-1} b / l_jj.  sx: max ncol doubles
// of dynamic LDS.
template <int NT>
__global__ __launch_bounds__(NT) void k_nd_invert(double *__restrict__ P, const int64_t *__restrict__ sn_ptr,
                                                  const int32_t *__restrict__ ncol, const int32_t *__restrict__ nrow,
                                                  const int64_t *__restrict__ voff) {
    extern __shared__ double sx[];
    const int i = blockIdx.x, tid = threadIdx.x;
    for (int64_t J = sn_ptr[i]; J < sn_ptr[i + 1]; ++J) {
        const int nJ = ncol[J], ld = nrow[J];
        double *PJ = P + voff[J];
        for (int j = nJ - 1; j >= 0; --j) {
            for (int r = j + 1 + tid; r < nJ; r += NT) sx[r] = PJ[int64_t(j) * ld + r];
            __syncthreads();
            const double ajj = 1.0 / PJ[int64_t(j) * ld + j];
            for (int r = j + 1 + tid; r < nJ; r += NT) {
                double acc = 0.0;
                for (int c = j + 1; c <= r; ++c) acc += PJ[int64_t(c) * ld + r] * sx[c];
                PJ[int64_t(j) * ld + r] = -ajj * acc;
            }
            __syncthreads();
            if (tid == 0) PJ[int64_t(j) * ld + j] = ajj;
            __syncthreads();
        }
    }
}

// Panels (FP64) to the solve layout in the factor's storage type, one
// workgroup per supernode.
template <typename T>
__global__ __launch_bounds__(256) void k_nd_split(const double *__restrict__ P, T *__restrict__ out,
                                                  const int32_t *__restrict__ ncol, const int32_t *__restrict__ nrow,
                                                  const int64_t *__restrict__ voff) {
    const int64_t J = blockIdx.x;
    const int nJ = ncol[J], ld = nrow[J], ns = ld - nJ;
    const double *src = P + voff[J];
    T *dst = out + voff[J];
    const int64_t cnt = int64_t(nJ) * ld;
    for (int64_t e = threadIdx.x; e < cnt; e += 256) {
        const int c = int(e / ld), p = int(e - int64_t(c) * ld);
        const int64_t at = p < nJ ? int64_t(c) * nJ + p : int64_t(nJ) * nJ + int64_t(c) * ns + (p - nJ);
        dst[at] = from_double<T>(src[e]);
    }
}

// Sum over aligned groups of G lanes (G a power of two up to 64); every lane
// of a group gets its group's sum.  The lanes of a group must be active
// together; the other groups of the wavefront may be inactive.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
    for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Lanes per item for one pass of the solve over `items` items holding
// `work` multiply-adds in total: the power of two (at least gmin, at most
// 64) that minimises the rounds of a 1024-thread workgroup times the
// per-item chain (multiply-adds per lane plus two per reduction step: a
// step's cross-lane exchange costs about two multiply-add loads, measured
// on the 128^3 workload: weights 0, 0.25, 1, 2 and 4 gave 1.84, 1.49, 1.45,
// 1.44 and 1.46 ms per launch).  The
// choice depends on the subdomain alone, not on the launch's workgroup
// size, so every launch configuration sums in the same order.
__device__ __forceinline__ int lanes_for(int items, int work, int gmin) {
    constexpr int NT = 1024;
    if (items <= 0) return gmin;
    const int avg = int((int64_t(work) + items - 1) / items);
    int best = gmin;
    float bc = 3.0e38f;
    for (int G = gmin; G <= 64; G <<= 1) {
        const int rounds = int((int64_t(items) * G + NT - 1) / NT);
        const float c = float(rounds) * (float((avg + G - 1) / G) + 2.0f * float(__builtin_ctz(G)));
        if (c < bc) {
            bc = c;
            best = G;
        }
    }
    return best;
}

// Exact local solve A_i^{-1} r_i with the supernodal factor (L L^T after
// the nested-dissection ordering), one workgroup per subdomain, the vector
// in LDS in the new numbering, gather and scatter fused (slot: blockIdx.y).
// The supernodes are numbered by height, so the rows, the supernodes and the
// struct entries of one height are consecutive and independent of each
// other.  Forward, by height from the leaves:
//   (1) every row of the height subtracts the products of its descendants'
//       struct parts that land on it (kept in w, one value per struct entry);
//   (2) every row takes its row of the inverted diagonal block times those;
//   (3) every struct entry of the height's supernodes gets the product of
//       its row of the struct part with the supernode's new values, into w.
// Backward, by height from the root:
//   (4) every column c of a supernode J subtracts the product of its struct
//       part with the final values of J's struct rows;
//   (5) then takes column c of the inverted diagonal block (the transposed
//       solve) against those.
// Each pass gives every item a group of lanes (lanes_for, from the pass's
// item and multiply-add counts) whose partial products are summed in a
// fixed order; the values of one load instruction are consecutive in memory
// across groups in (2) and (3), within a group in (4) and (5) (the solve
// layout above; plain loads, so that a line shared by neighbouring items
// stays in the caches between them).  The leaves (no gathers) take (2), and
// (4) with (5), one chunk of whole leaves per wavefront, a lane per row, in
// place in the vector: a wavefront's LDS reads of a pass are issued before
// its writes, and no other wavefront touches the chunk's rows, so the
// leaves need neither the pass-result buffer nor a workgroup barrier
// between (4) and (5).  The subdomain's supernode table and each row's
// supernode are copied to LDS first, so that an item's factor loads wait on
// one global load at most.  w: one vector of struct-entry length per slot
// (slot stride nst).  LDS: nd_lds_bytes(maxrows, maxt, maxsn, accumulator
// size) (gdsw_impl.hpp).
template <int NT, typename VT>
__global__ __launch_bounds__(NT) void k_nd_apply(
    const double *__restrict__ r, const int32_t *__restrict__ ov_idx, const int64_t *__restrict__ ov_ptr,
    const int32_t *__restrict__ iperm, const VT *__restrict__ L, const int64_t *__restrict__ sn_ptr,
    const int32_t *__restrict__ first, const int32_t *__restrict__ ncol, const int32_t *__restrict__ nrow,
    const int64_t *__restrict__ voff, const int64_t *__restrict__ st_ptr, const int32_t *__restrict__ st_row,
    const int32_t *__restrict__ st_sn, const int32_t *__restrict__ row_sn, const int64_t *__restrict__ rc_ptr,
    const int32_t *__restrict__ rc_w, const int64_t *__restrict__ lv_base, const int32_t *__restrict__ lv_ptr,
    const int4 *__restrict__ lv_info, const int64_t *__restrict__ ch_base, const int32_t *__restrict__ ch_row,
    const double *__restrict__ dscale, double *__restrict__ zloc, typename AccOf<VT>::type *__restrict__ w,
    int64_t nst, int maxrows, int maxt, int maxsn, Skip sk) {
    using AT = typename AccOf<VT>::type;
    const int slot = blockIdx.y, i = sk.sub_at(blockIdx.x);
    // (subdomains without levels take the band solve)
    if (sk.sub(i, slot) || lv_base[i + 1] == lv_base[i]) return;
    r += slot * sk.sl.n;
    zloc += slot * sk.sl.zl;
    extern __shared__ __align__(16) unsigned char smraw[];
    const int r4 = (maxrows + 3) / 4 * 4, t4 = (maxt + 3) / 4 * 4;
    AT *y = reinterpret_cast<AT *>(smraw);
    AT *t = y + r4;
    int4 *snt = reinterpret_cast<int4 *>(t + t4);
    int *stp = reinterpret_cast<int *>(snt + maxsn);
    int16_t *rsn = reinterpret_cast<int16_t *>(stp + maxsn + 1);
    const int64_t o = ov_ptr[i];
    const int ni = int(ov_ptr[i + 1] - o);
    const int64_t s0 = sn_ptr[i];
    const int nsn = int(sn_ptr[i + 1] - s0);
    const int64_t sb = st_ptr[s0], vb = voff[s0];
    AT *wi = w + slot * nst + sb;
    const VT *Li = L + vb;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = NT / 64;
    for (int J = tid; J <= nsn; J += NT) {
        stp[J] = int(st_ptr[s0 + J] - sb);
        if (J < nsn) snt[J] = make_int4(first[s0 + J], ncol[s0 + J], nrow[s0 + J], int(voff[s0 + J] - vb));
    }
    for (int l = tid; l < ni; l += NT) {
        rsn[l] = int16_t(row_sn[o + l] - s0);
        const int d = ov_idx[o + l];
        double x = r[d];
        if (dscale) x *= dscale[d];
        y[iperm[o + l]] = AT(x);
    }
    __syncthreads();
    const int64_t lb = lv_base[i], cb = ch_base[i];
    const int nlev = int(lv_base[i + 1] - lb) - 1, nch = int(ch_base[i + 1] - cb) - 1;
    for (int lev = 0; lev < nlev; ++lev) {
        const int R0 = lv_ptr[lb + lev], R1 = lv_ptr[lb + lev + 1];
        const int4 a = lv_info[lb + lev];
        const int T0 = a.x, T1 = lv_info[lb + lev + 1].x;
        if (lev == 0) {
            // (2) on the leaves, in place
            for (int ch = wv; ch < nch; ch += NW) {
                const int rr = ch_row[cb + ch] + lane;
                AT acc = 0;
                if (rr < ch_row[cb + ch + 1]) {
                    const int4 J = snt[rsn[rr]];
                    const int c0 = rr - J.x;
                    const VT *row = Li + J.w + c0;
#pragma unroll 4
                    for (int c = 0; c <= c0; ++c) acc += to_acc(row[int64_t(c) * J.y]) * y[J.x + c];
                }
                __builtin_amdgcn_wave_barrier();
                if (rr < ch_row[cb + ch + 1]) y[rr] = acc;
            }
        } else {
            // (1)
            for (int rr = R0 + tid; rr < R1; rr += NT) {
                AT acc = y[rr];
                const int64_t e1 = rc_ptr[o + rr + 1];
                for (int64_t e = rc_ptr[o + rr]; e < e1; ++e) acc -= wi[rc_w[e]];
                t[rr - R0] = acc;
            }
            __syncthreads();
            // (2)
            const int G = lanes_for(R1 - R0, a.y, 1), g = tid & (G - 1);
            for (int rr = R0 + tid / G; rr < R1; rr += NT / G) {
                const int4 J = snt[rsn[rr]];   // first, columns, panel rows, value offset
                const int c0 = rr - J.x;
                const VT *row = Li + J.w + c0;
                const AT *tJ = t + (J.x - R0);
                AT acc = 0;
#pragma unroll 4
                for (int c = g; c <= c0; c += G) acc += to_acc(row[int64_t(c) * J.y]) * tJ[c];
                acc = group_sum(acc, G);
                if (g == 0) y[rr] = acc;
            }
        }
        __syncthreads();
        // (3)
        {
            const int G = lanes_for(T1 - T0, a.z, 1), g = tid & (G - 1);
            for (int q = T0 + tid / G; q < T1; q += NT / G) {
                const int k0 = int(st_sn[sb + q] - s0);
                const int4 K = snt[k0];
                const int ns = K.z - K.y;
                const VT *row = Li + K.w + int64_t(K.y) * K.y + (q - stp[k0]);
                AT acc = 0;
#pragma unroll 4
                for (int k = g; k < K.y; k += G) acc += to_acc(row[int64_t(k) * ns]) * y[K.x + k];
                acc = group_sum(acc, G);
                if (g == 0) wi[q] = acc;
            }
        }
        __syncthreads();
    }
    for (int lev = nlev - 1; lev >= 1; --lev) {
        const int R0 = lv_ptr[lb + lev], R1 = lv_ptr[lb + lev + 1];
        const int4 a = lv_info[lb + lev];
        // (4)
        {
            const int G = lanes_for(R1 - R0, a.z, 8), g = tid & (G - 1);
            for (int rr = R0 + tid / G; rr < R1; rr += NT / G) {
                const int j0 = rsn[rr];
                const int4 J = snt[j0];
                const int ns = J.z - J.y;
                const VT *col = Li + J.w + int64_t(J.y) * J.y + int64_t(rr - J.x) * ns;
                const int32_t *srow = st_row + sb + stp[j0];
                AT acc = 0;
#pragma unroll 4
                for (int q = g; q < ns; q += G) acc += to_acc(col[q]) * y[srow[q]];
                acc = group_sum(acc, G);
                if (g == 0) t[rr - R0] = y[rr] - acc;
            }
        }
        __syncthreads();
        // (5)
        {
            const int G = lanes_for(R1 - R0, a.y, 8), g = tid & (G - 1);
            for (int rr = R0 + tid / G; rr < R1; rr += NT / G) {
                const int4 J = snt[rsn[rr]];
                const int c = rr - J.x;
                const VT *col = Li + J.w + int64_t(c) * J.y;
                const AT *tJ = t + (J.x - R0);
                AT acc = 0;
#pragma unroll 4
                for (int k = c + g; k < J.y; k += G) acc += to_acc(col[k]) * tJ[k];
                acc = group_sum(acc, G);
                if (g == 0) y[rr] = acc;
            }
        }
        __syncthreads();
    }
    // (4) and (5) on the leaves, in place
    for (int ch = wv; ch < nch; ch += NW) {
        const int rr = ch_row[cb + ch] + lane;
        const bool in = rr < ch_row[cb + ch + 1];
        int4 J = make_int4(0, 0, 0, 0);
        AT acc = 0;
        if (in) {
            const int j0 = rsn[rr];
            J = snt[j0];
            const int ns = J.z - J.y;
            const VT *col = Li + J.w + int64_t(J.y) * J.y + int64_t(rr - J.x) * ns;
            const int32_t *srow = st_row + sb + stp[j0];
#pragma unroll 4
            for (int q = 0; q < ns; ++q) acc += to_acc(col[q]) * y[srow[q]];
            acc = y[rr] - acc;
        }
        __builtin_amdgcn_wave_barrier();
        if (in) y[rr] = acc;
        __builtin_amdgcn_wave_barrier();
        acc = 0;
        if (in) {
            const int c = rr - J.x;
            const VT *col = Li + J.w + int64_t(c) * J.y;
#pragma unroll 4
            for (int k = c; k < J.y; ++k) acc += to_acc(col[k]) * y[J.x + k];
        }
        __builtin_amdgcn_wave_barrier();
        if (in) y[rr] = acc;
    }
    __syncthreads();
    for (int l = tid; l < ni; l += NT) {
        const int d = ov_idx[o + l];
        double v = double(y[iperm[o + l]]);
        if (dscale) v *= dscale[d];
        zloc[o + l] = v;
    }
}

}  // namespace gdsw

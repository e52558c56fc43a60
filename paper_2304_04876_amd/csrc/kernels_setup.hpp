// Device kernels of the numerical setup, phase (b) of the paper's solver
// structure (Sec. V-A): local matrix values, local factorisations, the
// energy-minimising extension of eq. (2), the coarse matrix A_0 = Phi^T A Phi
// and its inverse.
#pragma once

#include "kernels_common.hpp"

namespace gdsw {

// out[dst[p]] = val[src[p]] * (scale ? scale[row[src[p]]] * scale[col[src[p]]] : 1)
// (dst == nullptr: out[p]; src[p] < 0: a fill entry, 0).  Used to gather the
// local matrices A_i and A_{I_i I_i} from A, optionally symmetrically
// diagonally scaled.
__global__ void k_gather_vals(const double *__restrict__ val, const int64_t *__restrict__ src,
                              const int64_t *__restrict__ dst, double *__restrict__ out, int64_t cnt,
                              const double *__restrict__ scale, const int32_t *__restrict__ arow,
                              const int32_t *__restrict__ acol) {
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < cnt;
         p += int64_t(gridDim.x) * blockDim.x) {
        const int64_t s = src[p];
        double v = 0.0;
        if (s >= 0) {
            v = val[s];
            if (scale) v *= scale[arow[s]] * scale[acol[s]];
        }
        out[dst ? dst[p] : p] = v;
    }
}

// ---------------------------------------------------------------------------
// FastILU (Sec. V-B, iterative variant of the incomplete factorisation):
// the entries of L (unit lower, strictly lower part stored) and U on the
// local patterns are fixed points of
//     l_ij = (a_ij - sum_{m<j} l_im u_mj) / u_jj   (i > j)
//     u_ij =  a_ij - sum_{m<i} l_im u_mj           (i <= j)
// and a sweep evaluates every entry from the previous sweep's values (one
// thread per entry, product pairs precomputed in ascending m).  Start:
// l_ij = a_ij / a_jj, u_ij = a_ij.
__global__ void k_fastilu_start(const double *__restrict__ a, const int32_t *__restrict__ dpos,
                                double *__restrict__ v, int64_t ne) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= ne) return;
    const int32_t d = dpos[e];
    v[e] = d >= 0 ? a[e] / a[d] : a[e];
}

__global__ void k_fastilu_sweep(const double *__restrict__ a, const int64_t *__restrict__ fptr,
                                const int32_t *__restrict__ pairs, const int32_t *__restrict__ dpos,
                                const double *__restrict__ vold, double *__restrict__ vnew, int64_t ne) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= ne) return;
    double acc = a[e];
    for (int64_t q = fptr[e]; q < fptr[e + 1]; ++q) acc -= vold[pairs[2 * q]] * vold[pairs[2 * q + 1]];
    const int32_t d = dpos[e];
    vnew[e] = d >= 0 ? acc / vold[d] : acc;
}

// status[i] = 1 + a local row of subdomain i whose pivot is zero or not
// finite (after FastILU sweeps); 0 if there is none
__global__ void k_ilu_pivot_check(const int64_t *__restrict__ ov_ptr, const int64_t *__restrict__ lrowptr,
                                  const int32_t *__restrict__ ldiag, const double *__restrict__ v,
                                  int *__restrict__ status) {
    const int i = blockIdx.x;
    const int64_t o = ov_ptr[i], ni = ov_ptr[i + 1] - o;
    for (int64_t l = threadIdx.x; l < ni; l += blockDim.x) {
        const double u = v[lrowptr[o + l] + ldiag[o + l]];
        if (u == 0.0 || !isfinite(u)) atomicCAS(status + i, 0, int(1 + l));
    }
}

// scale[d] = 1 / sqrt(A[d,d])
__global__ void k_diag_scale(const double *__restrict__ val, const int64_t *__restrict__ adiag,
                             double *__restrict__ scale, int64_t n) {
    int64_t d = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (d < n) scale[d] = 1.0 / sqrt(val[adiag[d]]);
}

__global__ void k_fill_i32(int *__restrict__ x, int v, int n) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) x[p] = v;
}

__global__ void k_fill(double *__restrict__ x, double v, int64_t n) {
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < n;
         p += int64_t(gridDim.x) * blockDim.x)
        x[p] = v;
}

// ---------------------------------------------------------------------------
// ILU(0) of every A_i in its natural (ascending global dof) order, in place on
// the local CSR values; one workgroup per subdomain, rows of one level of the
// dependency DAG in parallel (level-set scheduling, Sec. V-B "Incomplete
// Local Solver").  Row-by-row form: for each k < l in row l (ascending),
// l_lk = a_lk / u_kk and a_lj -= l_lk u_kj for the j > k in both rows.
// status[i] = 1 + local row of a zero pivot.
__global__ void k_ilu0_factor(const int64_t *__restrict__ ov_ptr, const int64_t *__restrict__ lrowptr,
                              const int32_t *__restrict__ lcol, const int32_t *__restrict__ ldiag,
                              const int64_t *__restrict__ lvl_base, const int32_t *__restrict__ lvl_ptr,
                              const int32_t *__restrict__ lvl_rows, double *__restrict__ lval,
                              int *__restrict__ status) {
    const int i = blockIdx.x;
    const int64_t o = ov_ptr[i];
    const int64_t lb = lvl_base[i];
    const int nlev = int(lvl_base[i + 1] - lb) - 1;
    for (int L = 0; L < nlev; ++L) {
        const int beg = lvl_ptr[lb + L], end = lvl_ptr[lb + L + 1];
        for (int q = beg + threadIdx.x; q < end; q += blockDim.x) {
            const int l = lvl_rows[o + q];
            const int64_t p = o + l;
            const int64_t rs = lrowptr[p], re = lrowptr[p + 1];
            for (int64_t e = rs; e < re; ++e) {
                const int k = lcol[e];
                if (k >= l) break;
                const int64_t pk = o + k;
                const int64_t dk = lrowptr[pk] + ldiag[pk];
                const double lik = lval[e] / lval[dk];
                lval[e] = lik;
                int64_t a = dk + 1, f = e + 1;
                const int64_t ke = lrowptr[pk + 1];
                while (a < ke && f < re) {
                    const int ca = lcol[a], cf = lcol[f];
                    if (ca == cf) {
                        lval[f] -= lik * lval[a];
                        ++a;
                        ++f;
                    } else if (ca < cf) {
                        ++a;
                    } else {
                        ++f;
                    }
                }
            }
            if (lval[rs + ldiag[p]] == 0.0) atomicCAS(status + i, 0, 1 + l);
        }
        __syncthreads();
    }
}

// Packs the ILU(0) factors into the padded slot-major layout of the Jacobi
// sweeps: for row p of subdomain i (padded row R = ell_off[i] + l) slot s of
// the strictly lower part L at [s * ell_rows + R], of the strictly upper part
// scaled by the pivot (U_lj / U_ll) likewise, and 1 / U_ll.  Unused slots
// hold 0 with column 0.
// Slots of the register-resident ILU(0) sweeps: three L and three U entries
// per row; their local columns packed two per 32-bit word.
constexpr int ILU_KL = 3, ILU_KU = 3, ILU_CW = (ILU_KL + ILU_KU + 1) / 2;
// slot counts of the register-resident sweeps with phased L and U loads
// (ILU(k) with fill)
constexpr int ILU_KL2 = 6, ILU_KU2 = 6, ILU_CW2 = (ILU_KL2 + ILU_KU2 + 1) / 2;
// zeroed factor rows past the last subdomain's (the phased sweeps read up
// to workgroup size x rows per thread rows from a subdomain's first)
constexpr int64_t ILU_PAD_ROWS = 8192;

template <typename VT>
__global__ void k_ilu_pack(const int64_t *__restrict__ ov_ptr, const int64_t *__restrict__ ell_off,
                           const int64_t *__restrict__ lrowptr, const int32_t *__restrict__ lcol,
                           const int32_t *__restrict__ ldiag, const double *__restrict__ lval,
                           int64_t ell_rows, int KL, int KU, VT *__restrict__ Lv,
                           uint16_t *__restrict__ Lc, VT *__restrict__ Uv, uint16_t *__restrict__ Uc,
                           VT *__restrict__ dinv, uint32_t *__restrict__ Cp, int64_t cp_stride) {
    const int i = blockIdx.y;
    const int64_t o = ov_ptr[i], ni = ov_ptr[i + 1] - o;
    const int64_t npad = ell_off[i + 1] - ell_off[i];
    const int64_t l = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (l >= npad) return;
    const int64_t R = ell_off[i] + l;
    int sl = 0, su = 0;
    if (l < ni) {
        const int64_t p = o + l;
        const int64_t rs = lrowptr[p], re = lrowptr[p + 1];
        const double piv = lval[rs + ldiag[p]];
        for (int64_t e = rs; e < re; ++e) {
            const int c = lcol[e];
            if (c < l) {
                Lv[sl * ell_rows + R] = from_double<VT>(lval[e]);
                Lc[sl * ell_rows + R] = uint16_t(c);
                ++sl;
            } else if (c > l) {
                Uv[su * ell_rows + R] = from_double<VT>(lval[e] / piv);
                Uc[su * ell_rows + R] = uint16_t(c);
                ++su;
            }
        }
        dinv[R] = from_double<VT>(1.0 / piv);
    } else {
        dinv[R] = from_double<VT>(0.0);
    }
    for (; sl < KL; ++sl) {
        Lv[sl * ell_rows + R] = from_double<VT>(0.0);
        Lc[sl * ell_rows + R] = 0;
    }
    for (; su < KU; ++su) {
        Uv[su * ell_rows + R] = from_double<VT>(0.0);
        Uc[su * ell_rows + R] = 0;
    }
    // Cp != nullptr: the row's L then U columns again, two per 32-bit word
    // (low half first), (KL + KU + 1) / 2 words per row, for the
    // register-resident sweeps: the words of a row together (cp_stride 0),
    // or word w of every row at w * cp_stride (each phase of the phased
    // sweeps then reads only its own words)
    if (Cp) {
        const int cw = (KL + KU + 1) / 2;
        for (int w = 0; w < cw; ++w) {
            uint32_t v = 0;
            for (int h = 0; h < 2; ++h) {
                const int k = 2 * w + h;
                const uint32_t c = k < KL ? Lc[k * ell_rows + R] : (k < KL + KU ? Uc[(k - KL) * ell_rows + R] : 0u);
                v |= c << (16 * h);
            }
            Cp[cp_stride ? w * cp_stride + R : R * cw + w] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Banded Cholesky A = L L^T of one symmetric positive definite matrix per
// workgroup, in place in FP64.  Row-major band storage: row r holds columns
// r-b .. r at band[r*(b+1) + (c - r + b)]; the diagonal slot holds 1/L_rr.  Blocked right-looking algorithm
// with panels of NB columns: factor the diagonal block in LDS, solve the
// rows below it (at most b of them), then update the (at most b x b) window
// below the panel.  The fill of a banded Cholesky factor stays inside the
// band.  status[i] = 1 + row of the first non-positive pivot.
constexpr int CH_NB = 16;
constexpr int CH_LD = CH_NB + 1;   // padded LDS row stride (bank spread)

template <int NT>
__global__ __launch_bounds__(NT) void k_band_chol(double *__restrict__ band, const int64_t *__restrict__ off,
                                                  const int32_t *__restrict__ bwid,
                                                  const int64_t *__restrict__ rptr, int *__restrict__ status) {
    extern __shared__ double smem[];
    const int i = blockIdx.x;
    if (off[i + 1] == off[i]) return;   // no band (empty, or a supernodal subdomain)
    const int n = int(rptr[i + 1] - rptr[i]);
    const int b = bwid[i];
    const int64_t w = b + 1;
    double *L = band + off[i];
    double *sD = smem;                 // CH_NB x CH_LD
    double *sdg = sD + CH_NB * CH_LD;  // CH_NB
    double *sP = sdg + CH_NB;          // b x CH_LD
    const int tid = threadIdx.x;
    for (int k0 = 0; k0 < n; k0 += CH_NB) {
        const int kb = min(CH_NB, n - k0);
        // (a) diagonal block, left-looking by columns
        for (int e = tid; e < CH_NB * CH_NB; e += NT) {
            const int t = e / CH_NB, s = e % CH_NB;
            double v = 0.0;
            if (t < kb && s <= t && t - s <= b) v = L[int64_t(k0 + t) * w + (s - t + b)];
            sD[t * CH_LD + s] = v;
        }
        __syncthreads();
        for (int j = 0; j < kb; ++j) {
            const int t = j + tid;
            if (t < kb) {
                double v = sD[t * CH_LD + j];
                for (int s = 0; s < j; ++s) v -= sD[t * CH_LD + s] * sD[j * CH_LD + s];
                if (t == j) {
                    if (!(v > 0.0)) {
                        atomicCAS(status + i, 0, 1 + k0 + j);
                        v = 1.0;
                    }
                    sdg[j] = sqrt(v);
                } else {
                    sD[t * CH_LD + j] = v;
                }
            }
            __syncthreads();
            if (t > j && t < kb) sD[t * CH_LD + j] /= sdg[j];
            __syncthreads();
        }
        for (int e = tid; e < kb * kb; e += NT) {
            const int t = e / kb, s = e % kb;
            if (s <= t && t - s <= b)
                L[int64_t(k0 + t) * w + (s - t + b)] = (s == t) ? 1.0 / sdg[t] : sD[t * CH_LD + s];
        }
        // (b) rows below the diagonal block: P <- P L_D^{-T}
        const int rbeg = k0 + kb;
        const int rend = min(n, k0 + kb + b);
        const int m = max(0, rend - rbeg);
        for (int q = tid; q < m; q += NT) {
            const int r = rbeg + q;
            const int s0 = max(0, r - b - k0);
            double x[CH_NB];
#pragma unroll
            for (int s = 0; s < CH_NB; ++s) {
                double v = 0.0;
                if (s >= s0 && s < kb) {
                    v = L[int64_t(r) * w + (k0 + s - r + b)];
                    for (int t = 0; t < s; ++t) v -= x[t] * sD[s * CH_LD + t];   // x[t] = 0 for t < s0
                    v /= sdg[s];
                }
                x[s] = v;
            }
#pragma unroll
            for (int s = 0; s < CH_NB; ++s) {
                sP[q * CH_LD + s] = x[s];
                if (s >= s0 && s < kb) L[int64_t(r) * w + (k0 + s - r + b)] = x[s];
            }
        }
        __syncthreads();
        // (c) trailing window: A(r, c) -= P(r,:) . P(c,:), c <= r
        for (int e = tid; e < m * m; e += NT) {
            const int rq = e / m, cq = e % m;
            if (cq > rq) continue;
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < CH_NB; ++s) acc += sP[rq * CH_LD + s] * sP[cq * CH_LD + s];
            const int r = rbeg + rq, c = rbeg + cq;
            L[int64_t(r) * w + (c - r + b)] -= acc;
        }
        __syncthreads();
    }
}

// Partitioned inverse of the diagonal blocks of a band Cholesky factor
// (FP64, before any cast): the 64x64 diagonal block L_kk of rows k0 ..
// k0+kb-1 is replaced in place by X = L_kk^{-1} (lower triangular; its
// diagonal, 1/L_tt, is what the band already holds there), so that the
// triangle solves of the block become products with X.  Only for bands of
// at least BS_NB - 1, where the whole triangle lies inside the band.  One
// 64-thread workgroup per diagonal block (block q of subdomain i with
// blk_ptr[i] <= q < blk_ptr[i+1]); thread c forms column c of X by forward
// substitution, X(t, c) = -(1/L_tt) sum_{c <= s < t} L(t, s) X(s, c).
constexpr int BS_NB_INV = 64;
__global__ __launch_bounds__(64) void k_band_invert_diag(double *__restrict__ band, const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ bwid,
                                                         const int64_t *__restrict__ rptr,
                                                         const int64_t *__restrict__ blk_ptr, int np) {
    extern __shared__ double smem[];
    constexpr int NB = BS_NB_INV, LD = NB + 1;
    double *sT = smem;             // NB x LD: the block of L
    double *sX = smem + NB * LD;   // NB x LD: its inverse
    const int64_t q = blockIdx.x;
    int lo = 0, hi = np;   // subdomain with blk_ptr[i] <= q < blk_ptr[i+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (blk_ptr[mid] <= q) lo = mid; else hi = mid;
    }
    const int i = lo;
    const int b = bwid[i];
    if (b < NB - 1) return;   // (the host gives narrow bands no blocks)
    const int n = int(rptr[i + 1] - rptr[i]);
    const int k0 = int(q - blk_ptr[i]) * NB;
    const int kb = min(NB, n - k0);
    const int64_t w = b + 1;
    double *L = band + off[i];
    const int c = threadIdx.x;
    for (int e = c; e < NB * NB; e += 64) {
        const int t = e / NB, s2 = e % NB;
        sT[t * LD + s2] = (t < kb && s2 <= t) ? L[int64_t(k0 + t) * w + (s2 - t + b)] : 0.0;
    }
    __syncthreads();
    if (c < kb) {
        sX[c * LD + c] = sT[c * LD + c];
        for (int t = c + 1; t < kb; ++t) {
            double acc = 0.0;
            for (int s2 = c; s2 < t; ++s2) acc += sT[t * LD + s2] * sX[s2 * LD + c];
            sX[t * LD + c] = -acc * sT[t * LD + t];
        }
    }
    __syncthreads();
    for (int e = c; e < NB * NB; e += 64) {
        const int t = e / NB, s2 = e % NB;
        if (t < kb && s2 < t) L[int64_t(k0 + t) * w + (s2 - t + b)] = sX[t * LD + s2];
    }
}

// Casts a band (FP64) into the storage precision of the local factors.
template <typename VT>
__global__ void k_cast(const double *__restrict__ src, VT *__restrict__ dst, int64_t cnt) {
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < cnt;
         p += int64_t(gridDim.x) * blockDim.x)
        dst[p] = from_double<VT>(src[p]);
}

// ---------------------------------------------------------------------------
// Band triangular solves with one LDS vector: y <- (L L^T)^{-1} y, L in the
// band layout above (reciprocal diagonal).  Blocks of 64 rows, two barriers
// per block:
//   forward, step of block k: block k's contribution is subtracted from the
//   rows below it, 16 lanes per row reading the row's 64-value band segment
//   side by side, and the workgroup stages block k+1's triangle in LDS; then
//   wavefront 0 solves block k+1 (lane t = row t), broadcasting each solved
//   value with a lane read;
//   backward (L^T z = y) is the mirror image by columns: the entries above
//   block k get its contribution (column j of the block's rows: consecutive
//   threads, consecutive addresses), and wavefront 0 solves block k-1's
//   transposed triangle (lane t = column t).
constexpr int BS_NB = 64;
static_assert(BS_NB == BS_NB_INV, "the inverted diagonal blocks are the solve's blocks");

// Loads of band entries: non-temporal for 8-byte entries (each band is
// streamed once per pass in whole cache lines); 4- and 2-byte entries use
// plain loads, since a row's 64-entry segment then fills only part of a
// line and the rest of the line is read by the next load.
template <typename VT>
__device__ __forceinline__ VT band_ld(const VT *p) {
    if constexpr (sizeof(VT) == 8)
        return ld_once(p);
    else
        return *p;
}

// A band of width b holds whole 64x64 triangles, and so gets its diagonal
// blocks inverted (k_band_invert_diag), when b >= 63.  The choice depends
// on the subdomain alone, so a problem's results do not depend on what it
// is packed with; the solve kernels come in one instance per choice, each
// leaving the other kind's subdomains alone.
__host__ __device__ constexpr bool band_inverted(int b) { return b >= BS_NB - 1; }
constexpr int BS_LD = BS_NB + 1;


// sT(t, s) = L(k0+t, k0+s) for s < t, 1/L(k0+t, k0+t) for s = t (all threads)
template <typename VT, typename AT, int NT>
__device__ __forceinline__ void band_stage_triangle(const VT *__restrict__ L, int64_t w, int b, int k0, int kb,
                                                    AT *sT) {
#pragma unroll 4
    for (int e = threadIdx.x; e < BS_NB * BS_NB; e += NT) {
        const int t = e / BS_NB, s = e % BS_NB;
        AT v = 0;
        if (t < kb && s <= t && t - s <= b) v = to_acc(band_ld(&L[int64_t(k0 + t) * w + (s - t + b)]));
        sT[t * BS_LD + s] = v;
    }
}

// The same block solves with the inverted diagonal block staged (bands of at
// least BS_NB - 1): lane t forms row t of X y (forward) or of X^T y
// (backward) in one pass of products; entries outside the triangle are zero
// in the staging, and the clamp keeps the reads inside the block.
// For a whole block (kb = 64, every block but a subdomain's last) the
// vector entries sit at fixed offsets from a 16-byte aligned address (the
// solve's LDS vector starts 16-byte aligned and blocks start at multiples of
// 64 entries), so their broadcast reads merge into wide LDS reads.
template <typename AT>
__device__ __forceinline__ const AT *band_block_vec(const AT *y, int k0) {
    return static_cast<const AT *>(__builtin_assume_aligned(y + k0, 16));
}

template <typename AT>
__device__ __forceinline__ void band_block_fwd_inv(const AT *sT, AT *y, int k0, int kb, int lane) {
    const AT *row = sT + lane * BS_LD;
    AT acc = 0;
    if (kb == BS_NB) {
        const AT *yb = band_block_vec(y, k0);
#pragma unroll 8
        for (int s = 0; s < BS_NB; ++s) acc += row[s] * yb[s];
    } else {
#pragma unroll 8
        for (int s = 0; s < BS_NB; ++s) acc += row[s] * y[k0 + min(s, kb - 1)];
    }
    if (lane < kb) y[k0 + lane] = acc;
}

template <typename AT>
__device__ __forceinline__ void band_block_bwd_inv(const AT *sT, AT *y, int k0, int kb, int lane) {
    AT acc = 0;
    if (kb == BS_NB) {
        const AT *yb = band_block_vec(y, k0);
#pragma unroll 8
        for (int s = 0; s < BS_NB; ++s) acc += sT[s * BS_LD + lane] * yb[s];
    } else {
#pragma unroll 8
        for (int s = 0; s < BS_NB; ++s) acc += sT[s * BS_LD + lane] * y[k0 + min(s, kb - 1)];
    }
    if (lane < kb) y[k0 + lane] = acc;
}

// The staged triangle is zero in rows kb..63 (pivot included), so the steps
// s >= kb leave the lanes below kb unchanged: no per-step test, which lets
// the unrolled steps read their LDS entries eight at a time ahead of the
// dependent arithmetic.
template <typename AT>
__device__ __forceinline__ void band_block_fwd(const AT *sT, AT *y, int k0, int kb, int lane) {
    AT yt = lane < kb ? y[k0 + lane] : AT(0);
    const AT *row = sT + lane * BS_LD;
#pragma unroll 8
    for (int s = 0; s < BS_NB; ++s) {
        const AT l = row[s];
        if (lane == s) yt *= l;
        const AT ys = lane_read(yt, s);
        if (lane > s) yt -= l * ys;
    }
    if (lane < kb) y[k0 + lane] = yt;
}

template <typename AT>
__device__ __forceinline__ void band_block_bwd(const AT *sT, AT *y, int k0, int kb, int lane) {
    AT yt = lane < kb ? y[k0 + lane] : AT(0);
#pragma unroll 8
    for (int s = BS_NB - 1; s >= 0; --s) {
        const AT l = sT[s * BS_LD + lane];   // L(k0+s, k0+lane), or the reciprocal pivot at s = lane
        if (lane == s) yt *= l;
        const AT zs = lane_read(yt, s);
        if (lane < s) yt -= l * zs;
    }
    if (lane < kb) y[k0 + lane] = yt;
}

// The staging split in two, for the register budgets that allow it: the
// triangle's loads into registers, issued with the row or column updates of
// the same step so that both are in flight together, and the store into
// LDS after the updates.
template <int NT>
constexpr int tri_per_thread() { return (BS_NB * BS_NB + NT - 1) / NT; }

template <typename VT, typename AT, int NT>
__device__ __forceinline__ void band_load_triangle(const VT *__restrict__ L, int64_t w, int b, int k0, int kb,
                                                   AT (&tv)[tri_per_thread<NT>()]) {
#pragma unroll
    for (int c = 0; c < tri_per_thread<NT>(); ++c) {
        const int e = int(threadIdx.x) + c * NT;
        const int t = e / BS_NB, s = e % BS_NB;
        tv[c] = (e < BS_NB * BS_NB && t < kb && s <= t && t - s <= b) ? to_acc(band_ld(&L[int64_t(k0 + t) * w + (s - t + b)]))
                                                                      : AT(0);
    }
}

template <typename AT, int NT>
__device__ __forceinline__ void band_store_triangle(const AT (&tv)[tri_per_thread<NT>()], AT *sT) {
#pragma unroll
    for (int c = 0; c < tri_per_thread<NT>(); ++c) {
        const int e = int(threadIdx.x) + c * NT;
        if (e < BS_NB * BS_NB) sT[(e / BS_NB) * BS_LD + e % BS_NB] = tv[c];
    }
}

// The solve with its band loads one block step ahead (1024 threads).  A
// step first uses the entries loaded during the step before (the rows below
// the solved block, forward; the thread's column above it, backward),
// then issues the next step's entries and triangle into the same registers,
// so that those loads are in flight across the triangle solve and its two
// barriers instead of being waited for at the start of the next step.  Rows
// (columns) past the held ones are loaded in the step itself.  Every sum is
// formed in the same order as in the plain form below, so both give the
// same bits.
template <typename VT, typename AT, int NT, bool INV>
__device__ void band_llt_solve_ahead(const VT *__restrict__ L, int n, int b, AT *y, AT *sT) {
    constexpr bool F64 = sizeof(AT) == 8;
    constexpr int LPR = 16, RPI = NT / LPR, QN = BS_NB / LPR;
    static_assert(LPR == 16, "the row sums use rows of 16 lanes");
    constexpr int PF = F64 ? 4 : 6;      // forward: row groups of RPI rows held per step
    constexpr int RB = F64 ? 2 : 4;      // forward: row groups per pass past the held ones
    constexpr int BPF = F64 ? 16 : 32;   // backward: rows of the thread's first column held
    constexpr int G = F64 ? 8 : 32;      // backward: loads per group past the held rows
    const int64_t w = b + 1;
    const int tid = threadIdx.x, lane = tid & 63;
    const int sub = tid & (LPR - 1), rg = tid / LPR;
    const int nblk = (n + BS_NB - 1) / BS_NB;
    AT tv[tri_per_thread<NT>()];
    // ---- forward
    // v[it][q] = L(r, k0 + sub + 16 q) for the row r = k0 + 64 + it RPI + rg
    // below the block at k0 (zero outside the band and past the subdomain)
    AT v[PF][QN];
    auto load_rows = [&](int k0) {
        const int k1 = k0 + BS_NB, rend = min(n, k1 + b);
#pragma unroll
        for (int it = 0; it < PF; ++it) {
            const int r = k1 + it * RPI + rg;
            const int s0 = max(0, r - b - k0);
            const VT *row = L + int64_t(r) * w + (k0 - r + b);
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                const int s = sub + q * LPR;
                v[it][q] = (r < rend && s >= s0) ? to_acc(band_ld(&row[s])) : AT(0);
            }
        }
    };
    band_stage_triangle<VT, AT, NT>(L, w, b, 0, min(BS_NB, n), sT);
    __syncthreads();
    if (tid < 64) {
        if constexpr (INV) band_block_fwd_inv(sT, y, 0, min(BS_NB, n), lane);
        else band_block_fwd(sT, y, 0, min(BS_NB, n), lane);
    }
    if (nblk > 1) {
        load_rows(0);
        band_load_triangle<VT, AT, NT>(L, w, b, BS_NB, min(BS_NB, n - BS_NB), tv);
    }
    __syncthreads();
    for (int blk = 0; blk + 1 < nblk; ++blk) {
        const int k0 = blk * BS_NB, k1 = k0 + BS_NB, kb1 = min(BS_NB, n - k1);
        const int rend = min(n, k1 + b);
        AT yq[QN];
#pragma unroll
        for (int q = 0; q < QN; ++q) yq[q] = y[k0 + sub + q * LPR];
#pragma unroll
        for (int it = 0; it < PF; ++it) {
            const int r = k1 + it * RPI + rg;
            AT acc = 0;
#pragma unroll
            for (int q = 0; q < QN; ++q) acc += v[it][q] * yq[q];
            acc = row16_sum(acc);
            if (r < rend && sub == 0) y[r] -= acc;
        }
        for (int r0 = k1 + PF * RPI; r0 < rend; r0 += RB * RPI) {
            AT u[RB][QN];
#pragma unroll
            for (int it = 0; it < RB; ++it) {
                const int r = r0 + it * RPI + rg;
                const int s0 = max(0, r - b - k0);
                const VT *row = L + int64_t(r) * w + (k0 - r + b);
#pragma unroll
                for (int q = 0; q < QN; ++q) {
                    const int s = sub + q * LPR;
                    u[it][q] = (r < rend && s >= s0) ? to_acc(band_ld(&row[s])) : AT(0);
                }
            }
#pragma unroll
            for (int it = 0; it < RB; ++it) {
                const int r = r0 + it * RPI + rg;
                AT acc = 0;
#pragma unroll
                for (int q = 0; q < QN; ++q) acc += u[it][q] * yq[q];
                acc = row16_sum(acc);
                if (r < rend && sub == 0) y[r] -= acc;
            }
        }
        band_store_triangle<AT, NT>(tv, sT);
        if (blk + 2 < nblk) {   // the next step's rows and triangle
            load_rows(k1);
            band_load_triangle<VT, AT, NT>(L, w, b, k1 + BS_NB, min(BS_NB, n - k1 - BS_NB), tv);
        }
        __syncthreads();
        if (tid < 64) {
            if constexpr (INV) band_block_fwd_inv(sT, y, k1, kb1, lane);
            else band_block_fwd(sT, y, k1, kb1, lane);
        }
        __syncthreads();
    }
    // ---- backward
    // cv[s] = L(k0 + s, j) for the thread's first column j = max(0, k0 - b) + tid
    // above the block at k0 (zero outside the band)
    AT cv[BPF];
    auto load_col = [&](int k0) {
        const int kb = min(BS_NB, n - k0), j = max(0, k0 - b) + tid;
        const int smax = min(kb, j + b - k0 + 1);
        const VT *col = L + int64_t(k0) * w + (j - k0 + b);
#pragma unroll
        for (int s = 0; s < BPF; ++s) cv[s] = (j < k0 && s < smax) ? to_acc(band_ld(&col[int64_t(s) * (w - 1)])) : AT(0);
    };
    {
        const int k0 = (nblk - 1) * BS_NB, kb = n - k0;
        band_stage_triangle<VT, AT, NT>(L, w, b, k0, kb, sT);
        __syncthreads();
        if (tid < 64) {
            if constexpr (INV) band_block_bwd_inv(sT, y, k0, kb, lane);
            else band_block_bwd(sT, y, k0, kb, lane);
        }
        if (nblk > 1) {
            load_col(k0);
            band_load_triangle<VT, AT, NT>(L, w, b, k0 - BS_NB, BS_NB, tv);
        }
        __syncthreads();
    }
    for (int blk = nblk - 1; blk > 0; --blk) {
        const int k0 = blk * BS_NB, kb = min(BS_NB, n - k0);
        const int p0 = k0 - BS_NB;
        const int jbeg = max(0, k0 - b);
        {
            const int j = jbeg + tid;
            if (j < k0) {
                const int smax = min(kb, j + b - k0 + 1);
                const VT *col = L + int64_t(k0) * w + (j - k0 + b);
                // (the block's vector entries: at fixed offsets for a whole
                // block, clamped to the last row for the last one)
                auto col_sum = [&](auto yat) {
                    AT acc = 0;
#pragma unroll
                    for (int s = 0; s < BPF; ++s) acc += cv[s] * yat(s);
#pragma unroll 1
                    for (int g = BPF; g < BS_NB; g += G) {
                        AT u[G];
#pragma unroll
                        for (int q = 0; q < G; ++q)
                            u[q] = (g + q < smax) ? to_acc(band_ld(&col[int64_t(g + q) * (w - 1)])) : AT(0);
#pragma unroll
                        for (int q = 0; q < G; ++q) acc += u[q] * yat(g + q);
                    }
                    return acc;
                };
                const AT *yb = band_block_vec(y, k0);
                y[j] -= kb == BS_NB ? col_sum([&](int s) { return yb[s]; })
                                    : col_sum([&](int s) { return y[k0 + min(s, kb - 1)]; });
            }
        }
        // columns past the first NT (bands wider than the workgroup)
        for (int j = jbeg + tid + NT; j < k0; j += NT) {
            const int smax = min(kb, j + b - k0 + 1);
            const VT *col = L + int64_t(k0) * w + (j - k0 + b);
            AT acc = 0;
#pragma unroll 1
            for (int g = 0; g < BS_NB; g += G) {
                AT u[G];
#pragma unroll
                for (int q = 0; q < G; ++q)
                    u[q] = (g + q < smax) ? to_acc(band_ld(&col[int64_t(g + q) * (w - 1)])) : AT(0);
#pragma unroll
                for (int q = 0; q < G; ++q) acc += u[q] * y[k0 + min(g + q, kb - 1)];
            }
            y[j] -= acc;
        }
        band_store_triangle<AT, NT>(tv, sT);
        if (blk > 1) {   // the next step's column and triangle
            load_col(p0);
            band_load_triangle<VT, AT, NT>(L, w, b, p0 - BS_NB, BS_NB, tv);
        }
        __syncthreads();
        if (tid < 64) {
            if constexpr (INV) band_block_bwd_inv(sT, y, p0, BS_NB, lane);
            else band_block_bwd(sT, y, p0, BS_NB, lane);
        }
        __syncthreads();
    }
}

// INV: the diagonal blocks hold their inverses (band_inverted(b)), so each
// triangle solve is one product with the staged block.
// AHEAD: the form with the loads one step ahead (1024 threads: that
// register budget holds the extra entries without spills).
template <typename VT, typename AT, int NT, bool INV, bool AHEAD = false>
__device__ void band_llt_solve(const VT *__restrict__ L, int n, int b, AT *y, AT *sT) {
    if (n <= 0) return;   // an empty subdomain or interior (uniform over the workgroup)
    constexpr bool F64 = sizeof(AT) == 8;
    constexpr bool inv = INV;
    constexpr int G = F64 ? 8 : 32;   // loads in flight per thread and group (backward)
    // triangle loads overlapped with the updates where the register budget
    // holds the extra values (FP32 accumulation from 512 threads, FP64 at 1024)
    constexpr bool PREF = F64 ? NT >= 1024 : NT >= 512;
    if constexpr (AHEAD && PREF && NT >= 1024) {
        band_llt_solve_ahead<VT, AT, NT, INV>(L, n, b, y, sT);
        return;
    }
    const int64_t w = b + 1;
    const int tid = threadIdx.x, lane = tid & 63;
    const int nblk = (n + BS_NB - 1) / BS_NB;
    // ---- forward
    band_stage_triangle<VT, AT, NT>(L, w, b, 0, min(BS_NB, n), sT);
    __syncthreads();
    if (tid < 64) {
        if constexpr (inv) band_block_fwd_inv(sT, y, 0, min(BS_NB, n), lane);
        else band_block_fwd(sT, y, 0, min(BS_NB, n), lane);
    }
    __syncthreads();
    // rows below a solved block: 16 lanes per row, lane q takes the block's
    // columns q, q+16, q+32, q+48 (consecutive lanes, consecutive addresses)
    // and the 16 partial products are summed across the lanes
    constexpr int LPR = 16, RPI = NT / LPR;
    static_assert(LPR == 16, "the row sums use rows of 16 lanes");
    const int sub = tid & (LPR - 1), rg = tid / LPR;
    for (int blk = 0; blk + 1 < nblk; ++blk) {
        const int k0 = blk * BS_NB;
        const int k1 = k0 + BS_NB, kb1 = min(BS_NB, n - k1);
        const int rend = min(n, k1 + b);
        AT tv[tri_per_thread<NT>()];
        if constexpr (PREF) band_load_triangle<VT, AT, NT>(L, w, b, k1, kb1, tv);   // block k+1's triangle
        AT yq[BS_NB / LPR];
#pragma unroll
        for (int q = 0; q < BS_NB / LPR; ++q) yq[q] = y[k0 + sub + q * LPR];
        // RB row groups per pass: all their loads are issued before the sums
        constexpr int RB = sizeof(AT) == 8 ? 2 : 4;
        for (int r0 = k1; r0 < rend; r0 += RB * RPI) {
            AT v[RB][BS_NB / LPR];
#pragma unroll
            for (int it = 0; it < RB; ++it) {
                const int r = r0 + it * RPI + rg;
                const int s0 = max(0, r - b - k0);
                const VT *row = L + int64_t(r) * w + (k0 - r + b);
#pragma unroll
                for (int q = 0; q < BS_NB / LPR; ++q) {
                    const int s = sub + q * LPR;
                    v[it][q] = (r < rend && s >= s0) ? to_acc(band_ld(&row[s])) : AT(0);
                }
            }
#pragma unroll
            for (int it = 0; it < RB; ++it) {
                const int r = r0 + it * RPI + rg;
                AT acc = 0;
#pragma unroll
                for (int q = 0; q < BS_NB / LPR; ++q) acc += v[it][q] * yq[q];
                acc = row16_sum(acc);   // (LPR = 16 lanes per row)
                if (r < rend && sub == 0) y[r] -= acc;
            }
        }
        if constexpr (PREF) band_store_triangle<AT, NT>(tv, sT);
        else band_stage_triangle<VT, AT, NT>(L, w, b, k1, kb1, sT);
        __syncthreads();
        if (tid < 64) {
            if constexpr (inv) band_block_fwd_inv(sT, y, k1, kb1, lane);
            else band_block_fwd(sT, y, k1, kb1, lane);
        }
        __syncthreads();
    }
    // ---- backward
    {
        const int k0 = (nblk - 1) * BS_NB, kb = n - k0;
        band_stage_triangle<VT, AT, NT>(L, w, b, k0, kb, sT);
        __syncthreads();
        if (tid < 64) {
            if constexpr (inv) band_block_bwd_inv(sT, y, k0, kb, lane);
            else band_block_bwd(sT, y, k0, kb, lane);
        }
        __syncthreads();
    }
    for (int blk = nblk - 1; blk > 0; --blk) {
        const int k0 = blk * BS_NB, kb = min(BS_NB, n - k0);
        const int p0 = k0 - BS_NB;
        const int jbeg = max(0, k0 - b);
        AT tv[tri_per_thread<NT>()];
        if constexpr (PREF) band_load_triangle<VT, AT, NT>(L, w, b, p0, BS_NB, tv);   // block k-1's triangle
        for (int j = jbeg + tid; j < k0; j += NT) {
            const int smax = min(kb, j + b - k0 + 1);
            const VT *col = L + int64_t(k0) * w + (j - k0 + b);   // entry s at col[s * (w - 1)]
            AT acc = 0;
#pragma unroll 1
            for (int g = 0; g < BS_NB; g += G) {
                AT v[G];
#pragma unroll
                for (int q = 0; q < G; ++q) v[q] = (g + q < smax) ? to_acc(band_ld(&col[int64_t(g + q) * (w - 1)])) : AT(0);
#pragma unroll
                for (int q = 0; q < G; ++q) acc += v[q] * y[k0 + min(g + q, kb - 1)];
            }
            y[j] -= acc;
        }
        if constexpr (PREF) band_store_triangle<AT, NT>(tv, sT);
        else band_stage_triangle<VT, AT, NT>(L, w, b, p0, BS_NB, sT);
        __syncthreads();
        if (tid < 64) {
            if constexpr (inv) band_block_bwd_inv(sT, y, p0, BS_NB, lane);
            else band_block_bwd(sT, y, p0, BS_NB, lane);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Extension, eq. (2).  E_i = A_{I_i Gamma} Phi_Gamma(:, cols_i) is assembled
// one thread per interior row (couplings in CSR order), column-major
// n_Ii x k_i per subdomain at ext_off[i].
__global__ void k_ext_rhs(const double *__restrict__ Aval, const int64_t *__restrict__ int_ptr, int np,
                          const int64_t *__restrict__ ext_off, const int64_t *__restrict__ cpl_ptr,
                          const int64_t *__restrict__ cpl_apos, const int64_t *__restrict__ cpl_phi,
                          const int32_t *__restrict__ cpl_stride, const int32_t *__restrict__ cpl_rank,
                          const int32_t *__restrict__ cpl_slot, const int32_t *__restrict__ slotmap,
                          const double *__restrict__ phig, double *__restrict__ E, int64_t nint) {
    const int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (q >= nint) return;
    int lo = 0, hi = np;   // subdomain with int_ptr[i] <= q < int_ptr[i+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (int_ptr[mid] <= q) lo = mid; else hi = mid;
    }
    const int i = lo;
    const int64_t nr = int_ptr[i + 1] - int_ptr[i];
    const int64_t l = q - int_ptr[i];
    double *Ei = E + ext_off[i];
    for (int64_t e = cpl_ptr[q]; e < cpl_ptr[q + 1]; ++e) {
        const double a = Aval[cpl_apos[e]];
        const double *ph = phig + cpl_phi[e];
        const int st = cpl_stride[e], rk = cpl_rank[e], sl = cpl_slot[e];
        for (int j = 0; j < rk; ++j) Ei[int64_t(slotmap[sl + j]) * nr + l] += a * ph[int64_t(j) * st];
    }
}

// Phi_{I_i} = -A_{I_i I_i}^{-1} E_i, one workgroup per subdomain, one right
// hand side at a time through LDS, written into the subdomain's interior
// block of Phi.
template <int NT, bool INV>
__global__ __launch_bounds__(1024) void k_ext_solve(const double *__restrict__ iband,
                                                  const int64_t *__restrict__ iband_off,
                                                  const int32_t *__restrict__ ibw,
                                                  const int64_t *__restrict__ int_ptr,
                                                  const int64_t *__restrict__ scol_ptr,
                                                  const int64_t *__restrict__ ext_off,
                                                  const double *__restrict__ E,
                                                  const int32_t *__restrict__ sub_blk,
                                                  const int64_t *__restrict__ blk_val_off,
                                                  double *__restrict__ phi) {
    extern __shared__ __align__(16) double sxs[];   // (16-byte aligned: the band solve's block reads)
    double *smem = sxs;
    const int i = blockIdx.x;
    const int n = int(int_ptr[i + 1] - int_ptr[i]);
    const int k = int(scol_ptr[i + 1] - scol_ptr[i]);
    const int g = sub_blk[i];
    if (n == 0 || k == 0 || g < 0 || band_inverted(ibw[i]) != INV) return;
    double *y = smem;
    double *sT = smem + n;
    const double *L = iband + iband_off[i];
    for (int s = 0; s < k; ++s) {
        const double *e = E + ext_off[i] + int64_t(s) * n;
        for (int l = threadIdx.x; l < n; l += NT) y[l] = e[l];
        __syncthreads();
        band_llt_solve<double, double, NT, INV>(L, n, ibw[i], y, sT);
        double *out = phi + blk_val_off[g] + int64_t(s) * n;
        for (int l = threadIdx.x; l < n; l += NT) out[l] = -y[l];
        __syncthreads();
    }
}

// T1_i = E_i^T Phi_{I_i} (k_i x k_i), one thread per entry of one subdomain
__global__ void k_t1(const int64_t *__restrict__ int_ptr, const int64_t *__restrict__ scol_ptr,
                     const int64_t *__restrict__ ext_off, const double *__restrict__ E,
                     const int32_t *__restrict__ sub_blk, const int64_t *__restrict__ blk_val_off,
                     const double *__restrict__ phi, const int64_t *__restrict__ t1_off,
                     double *__restrict__ T1) {
    const int i = blockIdx.y;
    const int n = int(int_ptr[i + 1] - int_ptr[i]);
    const int k = int(scol_ptr[i + 1] - scol_ptr[i]);
    const int g = sub_blk[i];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (n == 0 || k == 0 || g < 0 || e >= k * k) return;
    const int a = e / k, bcol = e % k;
    const double *Ea = E + ext_off[i] + int64_t(a) * n;
    const double *Xb = phi + blk_val_off[g] + int64_t(bcol) * n;
    double acc = 0.0;
    for (int l = 0; l < n; ++l) acc += Ea[l] * Xb[l];
    T1[t1_off[i] + e] = acc;
}

// Interface-interface part of A_0: for every component pair (c, d) with
// couplings in A, the entries of Phi_Gc^T A_{cd} Phi_Gd, one thread per
// entry, couplings in a fixed order, into T2 (added into A_0 by target,
// k_a0_segments: components may share coarse columns).
__global__ void k_t2(const double *__restrict__ Aval, int npairs, const int32_t *__restrict__ pair_c,
                     const int32_t *__restrict__ pair_d, const int64_t *__restrict__ pair_off,
                     const int64_t *__restrict__ pair_eptr, const int64_t *__restrict__ pair_apos,
                     const int32_t *__restrict__ pair_lr_c, const int32_t *__restrict__ pair_lr_d,
                     const int32_t *__restrict__ comp_rank, const int64_t *__restrict__ phig_off,
                     const double *__restrict__ phig, double *__restrict__ T2, int64_t total) {
    const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= total) return;
    int lo = 0, hi = npairs;   // pair with pair_off[q] <= t < pair_off[q+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pair_off[mid] <= t) lo = mid; else hi = mid;
    }
    const int q = lo;
    const int c = pair_c[q], d = pair_d[q];
    const int rd = comp_rank[d];
    const int64_t loc = t - pair_off[q];
    const int a = int(loc / rd), bb = int(loc % rd);
    const int64_t nrc = (phig_off[c + 1] - phig_off[c]) / comp_rank[c];
    const int64_t nrd = (phig_off[d + 1] - phig_off[d]) / rd;
    const double *pc = phig + phig_off[c] + a * nrc;
    const double *pd = phig + phig_off[d] + bb * nrd;
    double acc = 0.0;
    for (int64_t e = pair_eptr[q]; e < pair_eptr[q + 1]; ++e)
        acc += pc[pair_lr_c[e]] * Aval[pair_apos[e]] * pd[pair_lr_d[e]];
    T2[t] = acc;
}

// A0[tgt] += sum of the subdomain contributions of the segment, ascending
// subdomain order
__global__ void k_a0_segments(const int64_t *__restrict__ seg_tgt, const int64_t *__restrict__ seg_ptr,
                              const int64_t *__restrict__ seg_src, const double *__restrict__ T1,
                              double *__restrict__ A0, int64_t nseg) {
    const int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (s >= nseg) return;
    double acc = 0.0;
    for (int64_t e = seg_ptr[s]; e < seg_ptr[s + 1]; ++e) acc += T1[seg_src[e]];
    A0[seg_tgt[s]] += acc;
}

// B = (A + A^T) / 2
__global__ void k_symmetrize(const double *__restrict__ A, double *__restrict__ B, int n) {
    const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= int64_t(n) * n) return;
    const int r = int(t / n), c = int(t % n);
    B[t] = 0.5 * (A[t] + A[int64_t(c) * n + r]);
}

// ---------------------------------------------------------------------------
// Inverse of the SPD coarse matrix by blocked Gauss-Jordan sweeps without
// pivoting (the pivots are Schur complements of an SPD matrix).  Sweeping
// block K of a symmetric matrix with P = A_KK^{-1}:
//   A_KK <- -P,  A_iK <- A_iK P,  A_Kj <- P A_Kj,  A_ij <- A_ij - A_iK P A_Kj;
// after all blocks the matrix holds -A^{-1}.
constexpr int GJ_NB = 32;
constexpr int GJ_LD = GJ_NB + 1;

// P = A_KK^{-1} in LDS by scalar sweeps, written to Pout (kb x kb)
__global__ __launch_bounds__(256) void k_gj_pivot(const double *__restrict__ A, int n, int k0, int kb,
                                                  double *__restrict__ Pout, int *__restrict__ status) {
    __shared__ double S[GJ_NB * GJ_LD];
    const int tid = threadIdx.x;
    for (int e = tid; e < kb * kb; e += 256) {
        const int r = e / kb, c = e % kb;
        S[r * GJ_LD + c] = A[int64_t(k0 + r) * n + (k0 + c)];
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        const double piv = S[j * GJ_LD + j];
        if (!(piv > 0.0)) {
            if (tid == 0) atomicCAS(status, 0, 1 + k0 + j);
            return;
        }
        const double p = 1.0 / piv;
        // all new values are computed from the old ones before any is stored
        double upd[4];
        int cnt = 0;
        for (int e = tid; e < kb * kb; e += 256, ++cnt) {
            const int rr = e / kb, cc = e % kb;
            double v = S[rr * GJ_LD + cc];
            const double aij = S[rr * GJ_LD + j], ajk = S[j * GJ_LD + cc];
            if (rr == j && cc == j) v = -p;
            else if (cc == j) v = aij * p;
            else if (rr == j) v = p * ajk;
            else v = v - aij * p * ajk;
            upd[cnt] = v;
        }
        __syncthreads();
        cnt = 0;
        for (int e = tid; e < kb * kb; e += 256, ++cnt) S[(e / kb) * GJ_LD + (e % kb)] = upd[cnt];
        __syncthreads();
    }
    for (int e = tid; e < kb * kb; e += 256) Pout[e] = -S[(e / kb) * GJ_LD + (e % kb)];
}

// W(i, :) = A(i, K) P for every row i (rows in K get 0)
__global__ void k_gj_panel(const double *__restrict__ A, int n, int k0, int kb, const double *__restrict__ P,
                           double *__restrict__ W) {
    __shared__ double sP[GJ_NB * GJ_NB];
    for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) sP[e] = P[e];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a[GJ_NB];
#pragma unroll
    for (int t = 0; t < GJ_NB; ++t) a[t] = (t < kb) ? A[int64_t(i) * n + k0 + t] : 0.0;
    const bool inK = (i >= k0 && i < k0 + kb);
    for (int s = 0; s < kb; ++s) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < GJ_NB; ++t)
            if (t < kb) acc += a[t] * sP[t * kb + s];
        W[int64_t(i) * GJ_NB + s] = inK ? 0.0 : acc;
    }
}

// A(i, j) -= W(i, :) . A(K, j) for i, j outside K; 64x64 tiles, 4x4 per thread
__global__ __launch_bounds__(256) void k_gj_update(double *__restrict__ A, int n, int k0, int kb,
                                                   const double *__restrict__ W) {
    __shared__ double sW[64 * GJ_LD];
    __shared__ double sK[GJ_NB * 65];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int tid = threadIdx.x;
    for (int e = tid; e < 64 * GJ_NB; e += 256) {
        const int r = e / GJ_NB, t = e % GJ_NB;
        const int i = i0 + r;
        sW[r * GJ_LD + t] = (i < n && t < kb) ? W[int64_t(i) * GJ_NB + t] : 0.0;
    }
    for (int e = tid; e < GJ_NB * 64; e += 256) {
        const int t = e / 64, c = e % 64;
        const int j = j0 + c;
        sK[t * 65 + c] = (j < n && t < kb) ? A[int64_t(k0 + t) * n + j] : 0.0;
    }
    __syncthreads();
    const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
    double acc[4][4] = {};
    for (int t = 0; t < kb; ++t) {
        double wv[4], kv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) wv[a] = sW[(tr + a) * GJ_LD + t];
#pragma unroll
        for (int c = 0; c < 4; ++c) kv[c] = sK[t * 65 + tc + c];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] += wv[a] * kv[c];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + tr + a;
        if (i >= n || (i >= k0 && i < k0 + kb)) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + tc + c;
            if (j >= n || (j >= k0 && j < k0 + kb)) continue;
            A[int64_t(i) * n + j] -= acc[a][c];
        }
    }
}

// A(i, K) = W(i, :), A(K, i) = W(i, :)^T (i outside K), A_KK = -P
__global__ void k_gj_fix(double *__restrict__ A, int n, int k0, int kb, const double *__restrict__ W,
                         const double *__restrict__ P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i >= k0 && i < k0 + kb) {
        const int r = i - k0;
        for (int t = 0; t < kb; ++t) A[int64_t(i) * n + k0 + t] = -P[r * kb + t];
        return;
    }
    for (int t = 0; t < kb; ++t) {
        const double v = W[int64_t(i) * GJ_NB + t];
        A[int64_t(i) * n + k0 + t] = v;
        A[int64_t(k0 + t) * n + i] = v;
    }
}

__global__ void k_negate(double *__restrict__ A, int64_t cnt) {
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < cnt;
         p += int64_t(gridDim.x) * blockDim.x)
        A[p] = -A[p];
}

}  // namespace gdsw

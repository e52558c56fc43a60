// Shared device helpers: precision conversions and deterministic reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <cstdint>

namespace gdsw {

using bf16 = __hip_bfloat16;
using fp16 = __half;

// arithmetic type for a storage type: FP64 stays FP64, everything else is
// accumulated in FP32
template <typename T> struct AccOf { using type = float; };
template <> struct AccOf<double> { using type = double; };

__device__ __forceinline__ double to_acc(double x) { return x; }
__device__ __forceinline__ float to_acc(float x) { return x; }
__device__ __forceinline__ float to_acc(fp16 x) { return __half2float(x); }
__device__ __forceinline__ float to_acc(bf16 x) { return __bfloat162float(x); }

template <typename T> __device__ __forceinline__ T from_double(double x);
template <> __device__ __forceinline__ double from_double<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_double<float>(double x) { return float(x); }
template <> __device__ __forceinline__ fp16 from_double<fp16>(double x) { return __float2half(float(x)); }
template <> __device__ __forceinline__ bf16 from_double<bf16>(double x) { return __float2bfloat16(float(x)); }

// Loads of data read once per launch (factor entries, matrix entries, the
// coarse inverse), marked non-temporal so that they do not displace data
// that later kernels of the same iteration read again from the caches (the
// coarse basis, the vectors).
template <typename T>
__device__ __forceinline__ T ld_once(const T *p) { return *p; }
template <>
__device__ __forceinline__ double ld_once<double>(const double *p) { return __builtin_nontemporal_load(p); }
template <>
__device__ __forceinline__ float ld_once<float>(const float *p) { return __builtin_nontemporal_load(p); }
template <>
__device__ __forceinline__ uint32_t ld_once<uint32_t>(const uint32_t *p) { return __builtin_nontemporal_load(p); }
template <>
__device__ __forceinline__ int32_t ld_once<int32_t>(const int32_t *p) { return __builtin_nontemporal_load(p); }
template <>
__device__ __forceinline__ int16_t ld_once<int16_t>(const int16_t *p) { return __builtin_nontemporal_load(p); }

// Lane moves without the LDS crossbar: DPP within rows of 16 lanes (quad
// permutations, mirrors of 8 and of 16 lanes), a swizzle across the halves
// of 32 lanes, and reads of one lane.  64-bit values move as two halves.
constexpr int DPP_QUAD_1032 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_2301 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;
constexpr int SWZ_XOR16 = 0x1F | (0x10 << 10);   // bit mode: and 0x1f, or 0, xor 0x10

template <int CTRL>
__device__ __forceinline__ float lane_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double lane_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_xor16(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), SWZ_XOR16));
}
__device__ __forceinline__ double lane_xor16(double v) {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), SWZ_XOR16);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), SWZ_XOR16);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_read(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double lane_read(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over each row of 16 lanes, with a fixed order; every lane of the row
// gets the same bits (each step adds a value and its partner's, and the two
// partners' sums commute).  All lanes of the wavefront must be active.
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
    v += lane_move<DPP_QUAD_1032>(v);
    v += lane_move<DPP_QUAD_2301>(v);
    v += lane_move<DPP_ROW_HALF_MIRROR>(v);
    v += lane_move<DPP_ROW_MIRROR>(v);
    return v;
}

// Sum over a wavefront with a fixed order (every lane gets it): rows of 16,
// pairs of rows, then the two halves of the wavefront.  All lanes active.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v = row16_sum(v);
    v += lane_xor16(v);
    return lane_read(v, 0) + lane_read(v, 32);
}

// Workgroup sum with a fixed order; `sh` must hold NT/64 values.  Every
// thread returns the total.  Contains two barriers.
template <typename T, int NT>
__device__ __forceinline__ T block_sum(T v, T *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    T t = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) t += sh[k];
    __syncthreads();
    return t;
}

// Right-hand-side slots: a handle may hold `ns` right-hand sides of every
// problem, all preconditioned with the one factored operator.  The vectors
// of the apply and the Krylov iteration hold the slots one after another
// (dof d of slot k at k n + d), and every buffer of per-slot intermediate
// results (local results, coarse partials, r_0, z_0 and its repetitions,
// the coarse part of the prolongation) is laid out the same way with the
// strides below.  Kernels over the operator's work items take the slot as
// blockIdx.y (or loop over the slots where the operator's values are held
// in registers).
struct Slots {
    int ns = 1;
    int64_t n = 0;       // dofs of one slot (the operator's dimension)
    int64_t zl = 0;      // local rows
    int64_t part = 0;    // coarse restriction partials
    int64_t n0 = 0;      // coarse columns
    int64_t cols = 0;    // repetitions of z_0 in block-column order
};

// Which parts of a launch to skip: a handle may pack several independent
// problems (block-diagonal A), each with `ns` slots; `flag[k nprob + p]` !=
// 0 means problem p in slot k is finished or idle and its subdomains,
// coarse blocks, coarse columns and dofs are left alone in that slot.
// flag == nullptr: nothing is skipped.
struct Skip {
    const int *flag = nullptr;
    const int32_t *sub_prob = nullptr;   // subdomain -> problem
    const int32_t *blk_prob = nullptr;   // coarse block -> problem
    const int32_t *cprob = nullptr;      // coarse column -> problem
    const int64_t *prob_ptr = nullptr;   // dof offsets of the problems
    int nprob = 1;
    Slots sl;
    // launch order of the local solves: workgroup b takes subdomain
    // order[b] (subdomains by decreasing size, so that the largest start
    // first and the hardware dispatcher, handing each free compute unit the
    // next workgroup, packs the smaller ones behind them); null: b itself
    const int32_t *order = nullptr;
    __device__ __forceinline__ int sub_at(int b) const { return order ? order[b] : b; }
    __device__ __forceinline__ bool sub(int i, int k = 0) const {
        return flag && flag[k * nprob + (nprob > 1 ? sub_prob[i] : 0)];
    }
    __device__ __forceinline__ bool blk(int g, int k = 0) const {
        return flag && flag[k * nprob + (nprob > 1 ? blk_prob[g] : 0)];
    }
    __device__ __forceinline__ bool col(int c, int k = 0) const {
        return flag && flag[k * nprob + (nprob > 1 ? cprob[c] : 0)];
    }
    // d: a dof of the operator (0 <= d < n), in slot k
    __device__ __forceinline__ bool dof(int64_t d, int k = 0) const {
        if (!flag) return false;
        if (nprob == 1) return flag[k];
        int lo = 0, hi = nprob;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (prob_ptr[mid] <= d) lo = mid; else hi = mid;
        }
        return flag[k * nprob + lo];
    }
};

}  // namespace gdsw

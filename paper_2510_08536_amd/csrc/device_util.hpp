// Device-side building blocks shared by the kernels: 64-lane wavefront
// reductions and scans, block reductions, the XCD-aware block remap and the
// deterministic re-summation of per-block partials.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rp_internal.hpp"

namespace rp {

// ---- wavefront (64 lanes) ------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma clang fp contract(off)
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) {
    const int lane = threadIdx.x & 63;
    for (int d = 1; d < 64; d <<= 1) {
        int32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Sum over a block of BLOCK threads, result valid in thread 0.  `red` holds
// BLOCK/64 values of shared memory.  Fixed shape, so the rounding is fixed.
template <typename T, int BLOCK>
__device__ __forceinline__ T block_sum(T v, T* red) {
#pragma clang fp contract(off)
    constexpr int NW = BLOCK / 64;
    __syncthreads();  // `red` may still be read from a previous call
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    T s = T(0);
    if (threadIdx.x == 0) {
        for (int i = 0; i < NW; ++i) s += red[i];
    }
    return s;
}

// Barrier for hand-offs through LDS only.  __syncthreads fences global
// memory too, which makes every wave wait for all of its outstanding global
// loads at the barrier; this one waits only for the wave's LDS (and scalar)
// accesses, so global loads issued before it stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---- XCD-aware block order -----------------------------------------------
// Workgroups are handed to the 8 XCDs round-robin (block b -> XCD b % 8).
// Remapping b to (b % 8) * per + b / 8 makes the logical blocks of one XCD
// consecutive, so neighbouring row groups (and the x entries they share) are
// worked on by one XCD and its L2.  gridDim.x must be a multiple of 8.
__device__ __forceinline__ int32_t xcd_block() {
    const int32_t per = (int32_t)(gridDim.x / N_XCD);
    return (int32_t)(blockIdx.x % N_XCD) * per + (int32_t)(blockIdx.x / N_XCD);
}

// Sum of partials[0..n), computed identically by every block of a kernel:
// thread t adds t, t + BLOCK, ... in order, then the fixed block tree.  The
// result is returned to every thread.  The partials come from an earlier
// kernel, so plain loads see them.
template <typename T, int BLOCK>
__device__ __forceinline__ T sum_partials_all(const T* partials, int32_t n, T* red) {
#pragma clang fp contract(off)
    __shared__ T bcast;
    T s = T(0);
    for (int32_t i = threadIdx.x; i < n; i += BLOCK) s += partials[i];
    const T b = block_sum<T, BLOCK>(s, red);
    if (threadIdx.x == 0) bcast = b;
    __syncthreads();
    return bcast;
}

}  // namespace rp

// Device-side building blocks shared by the kernels: 64-lane wavefront
// reductions and scans, block reductions, the XCD-aware block remap and the
// deterministic "last block finishes the reduction" protocol.
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

// ---- XCD-aware block order -----------------------------------------------
// Workgroups are handed to the 8 XCDs round-robin (block b -> XCD b % 8).
// Remapping b to (b % 8) * per + b / 8 gives each XCD one contiguous range of
// row groups, so the x entries a group gathers from its neighbours stay in
// that XCD's L2.  gridDim.x must be a multiple of 8.
__device__ __forceinline__ int32_t xcd_block() {
    const int32_t per = (int32_t)(gridDim.x / N_XCD);
    return (int32_t)(blockIdx.x % N_XCD) * per + (int32_t)(blockIdx.x / N_XCD);
}

// ---- coherent loads/stores for cross-block partials -----------------------
template <typename T>
__device__ __forceinline__ void store_partial(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T load_partial(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Arrival protocol: thread 0 of each block has stored its partial(s); returns
// true (block-uniform) in the block that arrives last, which then reads all
// partials in index order.  That block resets the counter for the next use.
__device__ __forceinline__ bool arrive_last(uint32_t* counter, uint32_t n_blocks) {
    __shared__ bool last;
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(counter, 1u);
        last = (prev == n_blocks - 1);
        if (last) __threadfence();
    }
    __syncthreads();
    return last;
}

// Deterministic sum of partials[0..n) by one block of BLOCK threads: thread t
// adds t, t+BLOCK, ... in order, then a fixed tree.  Result in thread 0.
template <typename T, int BLOCK>
__device__ __forceinline__ T sum_partials(const T* partials, int32_t n, T* red) {
#pragma clang fp contract(off)
    T s = T(0);
    for (int32_t i = threadIdx.x; i < n; i += BLOCK) s += load_partial(partials + i);
    __syncthreads();
    return block_sum<T, BLOCK>(s, red);
}

}  // namespace rp

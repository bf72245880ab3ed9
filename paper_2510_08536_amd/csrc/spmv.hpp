// CSR SpMV over one group of SPMV_BLOCK consecutive rows per workgroup.
//
// The group's nonzeros form one contiguous stretch of val/col.  The block
// streams that stretch with coalesced (non-temporal) loads, gathers x, and
// parks each product in LDS; then every thread sums its own row's products in
// column order.  With ~7 entries per row this keeps all 64 lanes busy on
// loads (a thread-per-row walk would stride the stream) and needs no
// cross-lane reduction.  Each product and each sum is rounded once, starting
// from 0, so the result is exactly that of the serial definition.
//
// Groups with more than SPMV_CAP nonzeros (rows far denser than a 7-point
// stencil) fall back to a direct per-row loop with the same arithmetic.
#pragma once

#include "device_util.hpp"

namespace rp {

template <typename T>
__device__ __forceinline__ T nt_load(const T* p) {
    return __builtin_nontemporal_load(p);
}

// Returns the row sum for row r0 + threadIdx.x (0 for threads past the group).
template <typename T>
__device__ __forceinline__ T spmv_group_row(const int32_t* __restrict__ row_ptr,
                                           const int32_t* __restrict__ col,
                                           const T* __restrict__ val, const T* __restrict__ x,
                                           int32_t r0, int32_t nr, T* lds) {
#pragma clang fp contract(off)
    const int t = threadIdx.x;
    const int32_t base = row_ptr[r0];
    const int32_t cnt = row_ptr[r0 + nr] - base;
    int32_t rs = 0, re = 0;
    if (t < nr) {
        rs = row_ptr[r0 + t];
        re = row_ptr[r0 + t + 1];
    }
    T s = T(0);
    if (cnt <= SPMV_CAP) {
        __syncthreads();  // the previous group may still be reading `lds`
        int32_t c[SPMV_UNROLL];
        T v[SPMV_UNROLL];
#pragma unroll
        for (int u = 0; u < SPMV_UNROLL; ++u) {
            const int32_t j = t + u * SPMV_BLOCK;
            if (j < cnt) {
                c[u] = nt_load(col + base + j);
                v[u] = nt_load(val + base + j);
            }
        }
#pragma unroll
        for (int u = 0; u < SPMV_UNROLL; ++u) {
            const int32_t j = t + u * SPMV_BLOCK;
            if (j < cnt) lds[j] = v[u] * x[c[u]];
        }
        __syncthreads();
        for (int32_t j = rs - base; j < re - base; ++j) s += lds[j];
    } else {
        for (int32_t j = rs; j < re; ++j) s += val[j] * x[col[j]];
    }
    return s;
}

// Row groups of block L (after xcd_block()) in a grid of G blocks: L, L + G,
// L + 2G, ...  At any moment the whole chip works on one window of G
// consecutive groups, and each XCD on a contiguous eighth of it, so the x
// entries a group gathers from neighbouring rows (a 3D stencil reaches a
// plane away) are still in that XCD's L2.
struct GroupRange {
    int32_t g0, n_groups, step;
};
__device__ __forceinline__ GroupRange block_groups(int32_t n_rows) {
    GroupRange r;
    r.n_groups = (int32_t)(((int64_t)n_rows + SPMV_BLOCK - 1) / SPMV_BLOCK);
    r.g0 = xcd_block();
    r.step = (int32_t)gridDim.x;
    return r;
}

}  // namespace rp

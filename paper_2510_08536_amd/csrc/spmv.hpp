// CSR SpMV over one group of SPMV_BLOCK consecutive rows per workgroup.
//
// Matrix stream: the group's nonzeros are one contiguous stretch of val/col.
// The block reads it with coalesced non-temporal loads of aligned pairs (two
// values / two column ids per lane), multiplies, parks each product in LDS,
// and every thread then sums its own row's products in column order.  Each
// product and each sum is rounded once, starting from 0, so the result is
// exactly that of the serial definition.
//
// x: by default every product's x entry is loaded straight from global
// memory, all of a thread's loads issued before the first product so they
// are in flight together.  Optionally (rp_plan_set_spmv_windows) x is staged
// in LDS windows instead: a 3D finite-volume stencil in a rank's natural
// cell order reads x at the row, at +-1 and +-nx (near the diagonal) and at
// +-nx*ny (a plane away), so the block copies a diagonal window
// x[r0 - H, r0 + 256 + H) and, per dominant long-range offset d found when
// the plan was built, x[r0 -+ d, r0 -+ d + 256) with coalesced loads; other
// columns are read from global memory.  On MI355X the direct loads measured
// faster (the HBM bytes are the same; the staging costs LDS, a barrier and
// occupancy), hence the default.  The arithmetic is the same either way.
#pragma once

#include "device_util.hpp"

namespace rp {

constexpr int XW_HALF = 64;                          // diagonal window half-width H
constexpr int XW_DIAG = SPMV_BLOCK + 2 * XW_HALF;    // diagonal window length
constexpr int SPMV_PAIRS = SPMV_CAP / 2;             // staged pairs per group

// window layout of a plan: NW = -1 no windows, 0 diagonal only, 1..2 plus
// that many +-d pairs (the offsets travel as kernel arguments)
struct XWin {
    int32_t d[2];
};

template <int NW>
struct XWinSize {
    static constexpr int value = NW < 0 ? 1 : XW_DIAG + 2 * NW * SPMV_BLOCK;
};

template <typename T>
__device__ __forceinline__ T nt_load(const T* p) {
    return __builtin_nontemporal_load(p);
}

template <typename T>
struct Pair;
template <>
struct Pair<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
typedef int32_t IdxPair __attribute__((ext_vector_type(2)));

// x[c] from the LDS windows of the group starting at row r0, else from global
template <typename T, int NW>
__device__ __forceinline__ T x_at(int32_t c, int32_t r0, const XWin& w, const T* xs, const T* __restrict__ x) {
    if (NW >= 0) {
        uint32_t o = (uint32_t)(c - (r0 - XW_HALF));
        if (o < (uint32_t)XW_DIAG) return xs[o];
#pragma unroll
        for (int k = 0; k < (NW > 0 ? NW : 0); ++k) {
            o = (uint32_t)(c - (r0 - w.d[k]));
            if (o < (uint32_t)SPMV_BLOCK) return xs[XW_DIAG + (2 * k) * SPMV_BLOCK + o];
            o = (uint32_t)(c - (r0 + w.d[k]));
            if (o < (uint32_t)SPMV_BLOCK) return xs[XW_DIAG + (2 * k + 1) * SPMV_BLOCK + o];
        }
    }
    return x[c];
}

// Row sum for row r0 + threadIdx.x (0 for threads past the group, nr rows).
// xs: XWinSize<NW> elements of LDS, lds: SPMV_CAP elements.  On return
// (NW >= 0) xs[XW_HALF + t] holds x of the thread's own row.
template <typename T, int NW>
__device__ __forceinline__ T spmv_group_row(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                           const T* __restrict__ val, const T* __restrict__ x, int32_t n,
                                           int32_t r0, int32_t nr, const XWin& w, T* xs, T* lds) {
#pragma clang fp contract(off)
    typedef typename Pair<T>::type VP;
    const int t = threadIdx.x;
    const int32_t base = row_ptr[r0];
    const int32_t end = row_ptr[r0 + nr];
    const int32_t al = base & ~1;                  // pairs start on an even index
    const int32_t npairs = (end - al + 1) >> 1;
    const bool staged = npairs <= SPMV_PAIRS;      // block-uniform
    int32_t rs = 0, re = 0;
    if (t < nr) {
        rs = row_ptr[r0 + t];
        re = row_ptr[r0 + t + 1];
    }
    __syncthreads();  // the previous group may still be reading xs / lds
    if (NW >= 0) {
        for (int i = t; i < XW_DIAG; i += SPMV_BLOCK) {
            const int32_t c = r0 - XW_HALF + i;
            xs[i] = (c >= 0 && c < n) ? x[c] : T(0);
        }
#pragma unroll
        for (int k = 0; k < (NW > 0 ? NW : 0); ++k) {
            const int32_t cm = r0 - w.d[k] + t, cp = r0 + w.d[k] + t;
            xs[XW_DIAG + (2 * k) * SPMV_BLOCK + t] = (cm >= 0 && cm < n) ? x[cm] : T(0);
            xs[XW_DIAG + (2 * k + 1) * SPMV_BLOCK + t] = (cp >= 0 && cp < n) ? x[cp] : T(0);
        }
    }
    constexpr int U = SPMV_PAIRS / SPMV_BLOCK;
    IdxPair c[U];
    VP v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        c[u] = IdxPair{0, 0};
        v[u] = VP{T(0), T(0)};
    }
    if (staged) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t k = t + u * SPMV_BLOCK;
            if (k < npairs) {
                if (2 * k + 2 <= end - al) {  // both entries inside [al, end): one 8/16-byte load
                    c[u] = nt_load(reinterpret_cast<const IdxPair*>(col + al) + k);
                    v[u] = nt_load(reinterpret_cast<const VP*>(val + al) + k);
                } else {                       // a lone last entry
                    c[u].x = col[al + 2 * k];
                    v[u].x = val[al + 2 * k];
                    c[u].y = 0;
                    v[u].y = T(0);
                }
            }
        }
    }
    if (NW < 0 && staged) {
        // direct x: issue all gathers before any product so they are in
        // flight together (lanes without entries hold column 0)
        T gx[2 * U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            gx[2 * u] = x[c[u].x];
            gx[2 * u + 1] = x[c[u].y];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t k = t + u * SPMV_BLOCK;
            if (k < npairs) {
                const int32_t p0 = al + 2 * k;
                if (p0 >= base) lds[p0 - base] = v[u].x * gx[2 * u];
                if (p0 + 1 < end) lds[p0 + 1 - base] = v[u].y * gx[2 * u + 1];
            }
        }
    }
    __syncthreads();  // windows staged
    if (NW >= 0 && staged) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t k = t + u * SPMV_BLOCK;
            if (k < npairs) {
                const int32_t p0 = al + 2 * k;
                if (p0 >= base) lds[p0 - base] = v[u].x * x_at<T, NW>(c[u].x, r0, w, xs, x);
                if (p0 + 1 < end) lds[p0 + 1 - base] = v[u].y * x_at<T, NW>(c[u].y, r0, w, xs, x);
            }
        }
    }
    __syncthreads();  // products staged (the direct path wrote them before the previous barrier)
    T s = T(0);
    if (staged) {
        for (int32_t j = rs - base; j < re - base; ++j) s += lds[j];
    } else {
        for (int32_t j = rs; j < re; ++j) s += val[j] * x_at<T, NW>(col[j], r0, w, xs, x);
    }
    return s;
}

// x of row i = r0 + threadIdx.x after spmv_group_row (from the diagonal window)
template <typename T, int NW>
__device__ __forceinline__ T own_x(int32_t i, const T* xs, const T* __restrict__ x) {
    if (NW >= 0) return xs[XW_HALF + threadIdx.x];
    return x[i];
}

// Row groups of block L (after xcd_block()) in a grid of G blocks: L, L + G,
// L + 2G, ...  At any moment the whole chip works on one window of G
// consecutive groups, and each XCD on a contiguous eighth of it.
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

// Expand CALL(NW) for the plan's window mode.
#define RP_DISPATCH_NW(nw, CALL)  \
    do {                          \
        switch (nw) {             \
        case -1: CALL(-1); break; \
        case 0: CALL(0); break;   \
        case 1: CALL(1); break;   \
        default: CALL(2); break;  \
        }                         \
    } while (0)

}  // namespace rp

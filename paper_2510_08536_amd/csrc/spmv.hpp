// CSR SpMV over one group of SPMV_BLOCK consecutive rows per workgroup.
//
// Two index forms, chosen per group when the plan is built:
//
// * offset-coded groups: a finite-volume stencil in a rank's natural cell
//   order couples each row i to i + o for a handful of offsets o (0, +-1,
//   +-nx, +-nx*ny, plus the jumps across processor interfaces).  When the
//   rows of a group use at most GOI_KMAX distinct offsets, the group keeps
//   its CSR values but replaces the column array by one ascending offset
//   table for the group and one bit mask per row (bit j: the row has column
//   i + off[j]).  Column order equals offset order, so the values stay in
//   CSR order.  The SpMV then reads no column indices: the x addresses come
//   straight from the row number, the table and the mask, so the x loads do
//   not wait for a load of col, and 4 bytes per entry less cross HBM.
// * plain CSR groups (everything else: scrambled numberings, rows with many
//   distinct offsets), described below.
//
// Both forms form every product and every row sum exactly as the serial
// definition does, so results are bit-identical whichever form runs.
//
// Matrix stream (CSR groups): the group's nonzeros are one contiguous stretch of val/col.
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
//
// Coded groups stage their values in LDS straight from memory (16-byte
// packs).  In FP64 they also stage the diagonal window x[r0 - 64, r0 + 320)
// for the taps within +-64 rows, and hold the x of only 8 taps in registers
// at a time (a 9th to 16th offset is summed after the first 8, in the same
// order), which keeps 7 waves per SIMD instead of 6.  FP32 measured faster
// without either and takes all 16 taps from memory in one pass.  Both
// precisions load the next group's metadata (offset count, value stretch,
// masks) while the current group's values load, and hand LDS over with
// barriers that do not wait for global loads (lds_barrier).
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

// Index arrays of the fused local block.  goi_k == nullptr: CSR everywhere.
struct SpmvIdx {
    const int32_t* row_ptr;    // [n+1]
    const int32_t* col;        // [nnz + SPMV_PAD]
    const int32_t* goi_k;      // [groups] offsets of a coded group, 0 = CSR group
    const int32_t* goi_off;    // [groups * GOI_KMAX] ascending col - row
    const uint16_t* goi_mask;  // [n] bit j: the row has column row + off[j]
};

// the index the kernels use for plan p
inline SpmvIdx spmv_idx(const rp_plan* p) {
    const bool coded = p->goi_on && p->coded_groups > 0;
    return SpmvIdx{p->d_row_ptr, p->d_col, coded ? p->d_goi_k : nullptr, p->d_goi_off, p->d_goi_mask};
}

template <typename T>
struct GroupRow {
    T s;         // row sum of the thread's row
    bool coded;  // the group ran offset-coded (no x windows staged)
    T xi;        // coded: x of the thread's row
};

// cache-policy bits of the direct-to-LDS loads: non-temporal (streamed once)
constexpr int SPMV_NT_AUX = 2;

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

// 16-byte packs of values (E entries) for the coded groups' value stream
template <typename T>
struct Pack;
template <>
struct Pack<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int E = 2;
};
template <>
struct Pack<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int E = 4;
};

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

// CSR group: row sum for row r0 + threadIdx.x (0 for threads past the
// group, nr rows).  xs: XWinSize<NW> elements of LDS, lds: SPMV_CAP
// elements.  On return (NW >= 0) xs[XW_HALF + t] holds x of the thread's
// own row.
template <typename T, int NW>
__device__ __forceinline__ T spmv_group_csr(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
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
    // Every lane loads a whole aligned pair; lanes past the stretch re-read
    // its last pair.  The loads thus carry no branch, and all of a thread's
    // loads are in flight together (a branch per load made the compiler wait
    // for each one before issuing the next).  The pair that straddles `end`
    // may touch one element past nnz: col and val hold SPMV_PAD zeroed
    // elements there, so the spare column is a valid index.  Entries outside
    // [base, end) are loaded but never used.
    {
        const int32_t last = npairs > 0 ? npairs - 1 : 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t k = min(t + u * SPMV_BLOCK, last);
            c[u] = nt_load(reinterpret_cast<const IdxPair*>(col + al) + k);
            v[u] = nt_load(reinterpret_cast<const VP*>(val + al) + k);
        }
    }
    if (NW < 0 && staged) {
        // direct x: issue all gathers before any product so they are in
        // flight together (every lane holds valid columns, see above)
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

// Metadata of one offset-coded group: its offset count K (0: a CSR group),
// its value stretch [base, end), and the thread's row mask.  The kernels load
// it one group ahead (spmv_group_row).  The offset table is not part of it:
// held a group ahead it cost enough scalar registers to spill them, and the
// SpMV measured slower than with the table loaded when the group starts.
struct CodedMeta {
    int32_t K, base, end;
    uint32_t m;
};

// The group-uniform values are read through the constant address space, so
// they are scalar loads into scalar registers (the index arrays are not
// written while an SpMV runs); the mask is a vector load.
typedef const __attribute__((address_space(4))) int32_t* ConstI32;

__device__ __forceinline__ void coded_meta_load(const SpmvIdx& ix, int32_t g, int32_t n, CodedMeta& c) {
    const int32_t r0 = g * SPMV_BLOCK, nr = min(SPMV_BLOCK, n - r0);
    c.K = ((ConstI32)ix.goi_k)[g];
    c.base = ((ConstI32)ix.row_ptr)[r0];
    c.end = ((ConstI32)ix.row_ptr)[r0 + nr];
    c.m = (int32_t)threadIdx.x < nr ? (uint32_t)ix.goi_mask[r0 + threadIdx.x] : 0u;
}

// Row groups of block L (after xcd_block()) in a grid of G blocks: L, L + G,
// L + 2G, ...  At any moment the whole chip works on one window of G
// consecutive groups, and each XCD on a contiguous eighth of it.
// meta: the first group's coded metadata, when the plan has coded groups.
struct GroupRange {
    int32_t g0, n_groups, step;
    CodedMeta meta;
};
__device__ __forceinline__ GroupRange block_groups(const SpmvIdx& ix, int32_t n_rows) {
    GroupRange r;
    r.n_groups = (int32_t)(((int64_t)n_rows + SPMV_BLOCK - 1) / SPMV_BLOCK);
    r.g0 = xcd_block();
    r.step = (int32_t)gridDim.x;
    r.meta.K = 0;
    if (ix.goi_k != nullptr && r.g0 < r.n_groups) coded_meta_load(ix, r.g0, n_rows, r.meta);
    return r;
}

// Offset-coded group g (K offsets): row sum for row r0 + threadIdx.x.
// lds: SPMV_CAP elements, 16-byte aligned.  The group's values are read as
// aligned 16-byte packs (2 doubles or 4 floats); when the plan is built, a
// group is coded only if its packs fit SPMV_CAP elements in both precisions.
template <typename T>
__device__ __forceinline__ GroupRow<T> spmv_group_coded(const SpmvIdx& ix, const T* __restrict__ val,
                                                      const T* __restrict__ x, int32_t n, int32_t r0,
                                                      int32_t nr, T* lds, CodedMeta& meta, int32_t g_next) {
#pragma clang fp contract(off)
    typedef typename Pack<T>::type VP;
    constexpr int E = Pack<T>::E;
    __shared__ int32_t wtot[SPMV_BLOCK / 64];
    const int t = threadIdx.x;
    // this group's metadata (loaded during the previous group) and offset table
    const int32_t K = meta.K, base = meta.base, end = meta.end;
    const uint32_t m = meta.m;
    int32_t off[GOI_KMAX];
    const ConstI32 offp = (ConstI32)ix.goi_off + (int64_t)(r0 / SPMV_BLOCK) * GOI_KMAX;
#pragma unroll
    for (int j = 0; j < GOI_KMAX; ++j) off[j] = offp[j];
    const int32_t al = base & ~(E - 1);            // packs start on a multiple of E
    const int32_t npk = (end - al + E - 1) / E;
    // FP64: the block's diagonal window x[r0 - XN, r0 + SPMV_BLOCK + XN) goes
    // to LDS, and taps with |offset| <= XN read it there instead of memory.
    // (FP32 runs slower with it and takes every tap from memory.)
    constexpr bool XWIN = sizeof(T) == 8;
    constexpr int XN = 64;
    __shared__ T xd[XWIN ? SPMV_BLOCK + 2 * XN : 1];
    T xa = T(0), xb = T(0);
    if constexpr (XWIN) {
        const int32_t e0 = r0 - XN + t, e1 = e0 + SPMV_BLOCK;
        if (e0 >= 0 && e0 < n) xa = x[e0];
        if (t < 2 * XN && e1 < n) xb = x[e1];
    }
    // the previous group's LDS reads are done before any load lands there
    // (global loads, such as the window's, stay in flight)
    lds_barrier();
    // the next group's metadata, in flight while this group's values load
    if (g_next >= 0) coded_meta_load(ix, g_next, n, meta);
    // the row's first entry: exclusive prefix of the row lengths (popcounts)
    const int32_t c = __popc(m);
    const int32_t inc = wave_incl_scan(c);
    if ((t & 63) == 63) wtot[t >> 6] = inc;
    // values: whole 16-byte packs straight from HBM into LDS.  The load
    // writes lane-linearly from a wave-uniform base, and pack k of the stretch
    // lands in LDS slot k.  Only lanes inside the stretch load (a wave wholly
    // past it issues nothing); the last pack may reach E - 1 elements past
    // `end` (SPMV_PAD).
    constexpr int U = SPMV_CAP / E / SPMV_BLOCK;
    typedef __attribute__((address_space(3))) void* LdsPtr;
    const int32_t wave0 = t & ~63;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (t + u * SPMV_BLOCK < npk)
            __builtin_amdgcn_global_load_lds((void*)(reinterpret_cast<const VP*>(val + al) + (t + u * SPMV_BLOCK)),
                                             (LdsPtr)(reinterpret_cast<VP*>(lds) + u * SPMV_BLOCK + wave0), 16, 0,
                                             SPMV_NT_AUX);
    // x of the present entries of the first KH taps, all issued before the
    // first use; taps KH.. (groups with more offsets) follow after the sums.
    // FP64 takes 8 at a time: the registers of all 16 would cost it a wave
    // per SIMD.  FP32 fits all 16 at full occupancy.
    constexpr int KH = XWIN ? GOI_KMAX / 2 : GOI_KMAX;
    T gx[KH];
    if constexpr (XWIN) {
#pragma unroll
        for (int j = 0; j < KH; ++j)
            gx[j] = (j < K && (off[j] < -XN || off[j] > XN) && ((m >> j) & 1u)) ? x[r0 + t + off[j]] : T(0);
        xd[t] = xa;
        if (t < 2 * XN) xd[t + SPMV_BLOCK] = xb;
    } else {
#pragma unroll
        for (int j = 0; j < KH; ++j) gx[j] = (j < K && ((m >> j) & 1u)) ? x[r0 + t + off[j]] : T(0);
    }
    // the packs of every wave must be in LDS before any wave reads them: wait
    // for all of this wave's loads, then the barrier
    __builtin_amdgcn_s_waitcnt(0);
    lds_barrier();
    if constexpr (XWIN) {
#pragma unroll
        for (int j = 0; j < KH; ++j)
            if (j < K && off[j] >= -XN && off[j] <= XN && ((m >> j) & 1u)) gx[j] = xd[XN + t + off[j]];
    }
    int32_t pos = inc - c + (base - al);
    for (int q = 0; q < (t >> 6); ++q) pos += wtot[q];
    T s = T(0);
#pragma unroll
    for (int j = 0; j < KH; ++j)
        if (j < K && ((m >> j) & 1u)) {
            s += lds[pos] * gx[j];
            ++pos;
        }
    if (KH < GOI_KMAX && K > KH) {
#pragma unroll
        for (int j = KH; j < GOI_KMAX; ++j) {
            T v = T(0);
            if (j < K && ((m >> j) & 1u)) {
                if (XWIN && off[j] >= -XN && off[j] <= XN) v = xd[XN + t + off[j]];
                else v = x[r0 + t + off[j]];
            }
            gx[j - KH] = v;
        }
#pragma unroll
        for (int j = KH; j < GOI_KMAX; ++j)
            if (j < K && ((m >> j) & 1u)) {
                s += lds[pos] * gx[j - KH];
                ++pos;
            }
    }
    if constexpr (XWIN) return GroupRow<T>{s, true, xd[XN + t]};
    return GroupRow<T>{s, true, t < nr ? x[r0 + t] : T(0)};
}

// Row sum of row g * SPMV_BLOCK + threadIdx.x in the form chosen for group g.
// gr carries the coded groups' metadata one group ahead: gr.meta describes
// group g on entry and group g + gr.step on return.
template <typename T, int NW>
__device__ __forceinline__ GroupRow<T> spmv_group_row(const SpmvIdx& ix, const T* __restrict__ val,
                                                     const T* __restrict__ x, int32_t n, int32_t g, int32_t nr,
                                                     const XWin& w, T* xs, T* lds, GroupRange& gr) {
    const int32_t r0 = g * SPMV_BLOCK;
    if (ix.goi_k != nullptr) {
        const int32_t g_next = g + gr.step < gr.n_groups ? g + gr.step : -1;
        if (gr.meta.K > 0) return spmv_group_coded<T>(ix, val, x, n, r0, nr, lds, gr.meta, g_next);
        const T s = spmv_group_csr<T, NW>(ix.row_ptr, ix.col, val, x, n, r0, nr, w, xs, lds);
        if (g_next >= 0) coded_meta_load(ix, g_next, n, gr.meta);
        return GroupRow<T>{s, false, T(0)};
    }
    return GroupRow<T>{spmv_group_csr<T, NW>(ix.row_ptr, ix.col, val, x, n, r0, nr, w, xs, lds), false, T(0)};
}

// x of row i = r0 + threadIdx.x after spmv_group_row (kept by the coded
// form; from the diagonal window when the group ran in CSR form with windows)
template <typename T, int NW>
__device__ __forceinline__ T own_x(int32_t i, const GroupRow<T>& gr, const T* xs, const T* __restrict__ x) {
    if (gr.coded) return gr.xi;
    if (NW >= 0) return xs[XW_HALF + threadIdx.x];
    return x[i];
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

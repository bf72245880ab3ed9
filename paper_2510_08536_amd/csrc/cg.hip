// Jacobi-preconditioned CG (the CG pressure solve of Sec. 4, M = diag(A)) and
// the two mixed-precision forms built on it.
//
// Iteration k is three kernels; all scalars stay on the device:
//   K1  q = A p                      partials of (p, q)
//   K2  alpha = rz_k / (p, q)        r -= alpha q;
//                                    partials of (r, M^-1 r) and (r, r)
//   K3  x += alpha p; stop tests, beta = rz_{k+1} / rz_k, p = M^-1 r + beta p
// (x moves in K3, which reads p anyway: one pass over p less per iteration)
// Small systems run K3 of iteration k and K1 of iteration k + 1 as one
// kernel (cg_update_xp_spmv), two launches per iteration with the same
// results bit for bit.
// Each kernel starts by adding up the previous kernel's per-block partials
// (every block the same sum, in index order), so reductions need no atomics,
// no fences and no extra launches, and reruns are bit-identical.  The
// iteration number k is a kernel argument; rz is kept in a ring indexed by
// it, because block 0 of K3 stores rz_{k+1} while other blocks still read
// rz_k.  Block 0 also records the state the host reads between chunks of
// iterations.  A stop decision is taken identically by every block, and
// kernels enqueued after a stop return at entry, so the iteration count does
// not depend on how many iterations the host enqueues per chunk.
//
// Ordering rule for the device state: the blocks of one launch may run in
// any order, and a block may start after block 0 has finished.  So a field
// that block 0 writes in a launch is read at entry by the same launch only
// where the outcome cannot differ: the writing path does no vector work, and
// every block reaches it from the same sums (the breakdown and stop paths of
// K2 and of the BiCGStab kernels).  K3 still moves x on its stop path, so it
// is gated on `kk`, which only K2 writes (the iteration K2 completed, -1 if
// K2 did nothing); BiCGStab's last kernel gates its half step on `half_k`,
// which only the kernel before it writes.
//
// Stop test: ||r||^2 <= tol^2 ||b||^2 on the recurrence residual, then
// confirmed on b - A x; a failed confirmation restarts CG from the current x.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>

#include "spmv.hpp"

namespace rp {

// cg_loop.hip: the iterations k0 .. min(k_end, budget) in one cooperative
// launch; *ran = false when the device cannot hold the grid at once
template <typename T>
int launch_cg_loop(rp_plan* p, int32_t n, const SpmvIdx& ix, const T* val, const T* dinv, T* x, T* r, T* pv, T* q,
                   CgState<T>* st, int32_t k0, int32_t k_end, hipStream_t s, bool* ran);

namespace {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// r = b - A x (x = 0 when XZERO, and then x is cleared); with W32 also
// r32 = RNE(r).  Partials of (r, r) -> PART_A and (b, b) -> PART_B.
template <typename T, bool XZERO, bool W32, int NW>
__global__ void __launch_bounds__(SPMV_BLOCK)
residual_kernel(int32_t n, SpmvIdx ix, const T* __restrict__ val, T* __restrict__ x, const T* b, T* r,
                float* r32, T* __restrict__ part, XWin w) {
#pragma clang fp contract(off)
    __shared__ __align__(16) T lds[XZERO ? 2 : SPMV_CAP];
    __shared__ T xs[XZERO ? 1 : XWinSize<NW>::value];
    __shared__ T red[SPMV_BLOCK / 64];
    T prr = T(0), pbb = T(0);
    GroupRange gr = block_groups(ix, n);
    for (int32_t g = gr.g0; g < gr.n_groups; g += gr.step) {
        const int32_t r0 = g * SPMV_BLOCK;
        const int32_t nr = min(SPMV_BLOCK, n - r0);
        T s = T(0);
        if (!XZERO) s = spmv_group_row<T, NW>(ix, val, x, n, g, nr, w, xs, lds, gr).s;
        if ((int32_t)threadIdx.x < nr) {
            const int32_t i = r0 + threadIdx.x;
            const T bi = b[i];
            const T ri = bi - s;
            if (XZERO) x[i] = T(0);
            r[i] = ri;
            if (W32) r32[i] = (float)ri;
            prr += ri * ri;
            pbb += bi * bi;
        }
    }
    const T brr = block_sum<T, SPMV_BLOCK>(prr, red);
    const T bbb = block_sum<T, SPMV_BLOCK>(pbb, red);
    if (threadIdx.x == 0) {
        const int32_t L = xcd_block();
        part[PART_A + L] = brr;
        part[PART_B + L] = bbb;
    }
}

// p = M^-1 r; partials of (r, M^-1 r) -> PART_RZ
template <typename T>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_start_p(int32_t n, const T* __restrict__ r, const T* __restrict__ dinv, T* __restrict__ p,
           T* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ T red[VEC_BLOCK / 64];
    T prz = T(0);
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        const T ri = r[i];
        const T zi = dinv[i] * ri;
        p[i] = zi;
        prz += ri * zi;
    }
    const T b = block_sum<T, VEC_BLOCK>(prz, red);
    if (threadIdx.x == 0) part[PART_RZ + blockIdx.x] = b;
}

// partials of (r, M^-1 r) -> PART_RZ and (r, r) -> PART_RR for a replaced residual
template <typename T>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_rz_rr(int32_t n, const T* __restrict__ r, const T* __restrict__ dinv, T* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ T red[VEC_BLOCK / 64];
    T prz = T(0), prr = T(0);
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        const T ri = r[i];
        prz += ri * (dinv[i] * ri);
        prr += ri * ri;
    }
    const T b1 = block_sum<T, VEC_BLOCK>(prz, red);
    const T b2 = block_sum<T, VEC_BLOCK>(prr, red);
    if (threadIdx.x == 0) {
        part[PART_RZ + blockIdx.x] = b1;
        part[PART_RR + blockIdx.x] = b2;
    }
}

enum : int32_t { FIN_START = 0, FIN_RESIDUAL = 1 };

// one block.  FIN_RESIDUAL: rr_true, bb from a residual_kernel.
// FIN_START: additionally (re)start CG at iteration k from that residual and
// cg_start_p's (r, z): thresh = tol2 * bb, pause_thresh = pause_frac2 * rr.
template <typename T>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_finalize(int32_t mode, int32_t k, int32_t max_iter, T tol2, T pause_frac2, int32_t g_spmv, int32_t g_vec,
            const T* __restrict__ part, CgState<T>* st) {
#pragma clang fp contract(off)
    __shared__ T red[VEC_BLOCK / 64];
    const T rr = sum_partials_all<T, VEC_BLOCK>(part + PART_A, g_spmv, red);
    const T bb = sum_partials_all<T, VEC_BLOCK>(part + PART_B, g_spmv, red);
    T rz = T(0);
    if (mode == FIN_START) rz = sum_partials_all<T, VEC_BLOCK>(part + PART_RZ, g_vec, red);
    if (threadIdx.x != 0) return;
    st->rr_true = rr;
    st->bb = bb;
    if (mode != FIN_START) return;
    const T thresh = tol2 * bb;
    st->thresh = thresh;
    st->rz[k & 3] = rz;
    st->rr = rr;
    st->rr_ref = rr;
    st->pause_frac2 = pause_frac2;
    st->pause_thresh = pause_frac2 * rr;
    st->iter = k;
    st->max_iter = max_iter;
    int32_t d = CG_RUNNING;
    if (bb == T(0)) d = CG_ZERO_RHS;
    else if (rr <= thresh) d = CG_CONVERGED;
    else if (!(rz > T(0)) || !isfinite(rz)) d = CG_BREAKDOWN;
    st->done = d;
}

// K1: q = A p; partials of (p, q) -> PART_A
template <typename T, int NW>
__global__ void __launch_bounds__(SPMV_BLOCK)
cg_spmv_pq(int32_t n, SpmvIdx ix, const T* __restrict__ val, const T* __restrict__ p, T* __restrict__ q,
           T* __restrict__ part, const CgState<T>* st, XWin w) {
#pragma clang fp contract(off)
    if (st->done != CG_RUNNING || st->iter >= st->max_iter) return;
    __shared__ __align__(16) T lds[SPMV_CAP];
    __shared__ T xs[XWinSize<NW>::value];
    __shared__ T red[SPMV_BLOCK / 64];
    T ppq = T(0);
    GroupRange gr = block_groups(ix, n);
    for (int32_t g = gr.g0; g < gr.n_groups; g += gr.step) {
        const int32_t r0 = g * SPMV_BLOCK;
        const int32_t nr = min(SPMV_BLOCK, n - r0);
        const GroupRow<T> gr_ = spmv_group_row<T, NW>(ix, val, p, n, g, nr, w, xs, lds, gr);
        if ((int32_t)threadIdx.x < nr) {
            const int32_t i = r0 + threadIdx.x;
            q[i] = gr_.s;
            ppq += own_x<T, NW>(i, gr_, xs, p) * gr_.s;
        }
    }
    const T b = block_sum<T, SPMV_BLOCK>(ppq, red);
    if (threadIdx.x == 0) part[PART_A + xcd_block()] = b;
}

// K2: alpha = rz_k / (p, q); r -= alpha q; partials of (r, M^-1 r) ->
// PART_RZ (RZ: Jacobi M) and (r, r) -> PART_RR.  x moves in K3, which reads
// p anyway.  Without RZ the preconditioner runs after this kernel and writes
// the (r, z) partials itself.
template <typename T, bool RZ = true>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_update_r(int32_t n, int32_t k_arg, int32_t g_spmv, T* __restrict__ r, const T* __restrict__ q,
            const T* __restrict__ dinv, T* __restrict__ part, CgState<T>* st) {
#pragma clang fp contract(off)
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    // K3 runs only if kk names its iteration, so every path that does no
    // update leaves kk = -1
    if (st->done != CG_RUNNING) {
        if (lead) st->kk = -1;
        return;
    }
    // iteration number: the argument, or (replayed graphs) the device state,
    // which only K3 and the finalize kernel write
    const int32_t k = k_arg >= 0 ? k_arg : st->iter;
    if (k >= st->max_iter) {
        if (lead) st->kk = -1;
        return;
    }
    __shared__ T red[VEC_BLOCK / 64];
    const T pq = sum_partials_all<T, VEC_BLOCK>(part + PART_A, g_spmv, red);
    if (!(pq > T(0)) || !isfinite(pq)) {
        if (lead) {
            st->pq = pq;
            st->iter = k;
            st->kk = -1;
            st->done = CG_BREAKDOWN;
        }
        return;
    }
    const T a = st->rz[k & 3] / pq;
    T prz = T(0), prr = T(0);
    const int32_t di = gridDim.x * VEC_BLOCK;
    int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x;
    // K2 sweeps the rows from the top down (element e = n - 1 - i), K1 and K3
    // from the bottom up: each kernel then starts on the lines its
    // predecessor touched last, which are still in the 256 MB memory-side
    // cache.  U of the thread's grid-stride elements per trip, all loads
    // first; the sums take the elements in the loop's order.
    constexpr int U = vec_unroll_r<T>();
    for (; (int64_t)i + (int64_t)(U - 1) * di < n; i += U * di) {
        T rv[U], qv[U], dv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t e = n - 1 - (i + u * di);
            rv[u] = r[e];
            qv[u] = q[e];
            dv[u] = RZ ? dinv[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t e = n - 1 - (i + u * di);
            const T ri = rv[u] - a * qv[u];
            r[e] = ri;
            if (RZ) {
                const T zi = dv[u] * ri;
                prz += ri * zi;
            }
            prr += ri * ri;
        }
    }
    for (; i < n; i += di) {
        const int32_t e = n - 1 - i;
        const T ri = r[e] - a * q[e];
        r[e] = ri;
        if (RZ) {
            const T zi = dinv[e] * ri;
            prz += ri * zi;
        }
        prr += ri * ri;
    }
    const T b1 = RZ ? block_sum<T, VEC_BLOCK>(prz, red) : T(0);
    const T b2 = block_sum<T, VEC_BLOCK>(prr, red);
    if (threadIdx.x == 0) {
        if (RZ) part[PART_RZ + blockIdx.x] = b1;
        part[PART_RR + blockIdx.x] = b2;
    }
    if (lead) {
        st->pq = pq;
        st->alpha = a;
        st->kk = k;
    }
}

// K3: x += alpha p (K2's alpha); stop tests on (r, r); unless stopping,
// beta = rz_{k+1} / rz_k and p = M^-1 r + beta p.  x uses the old p, exactly
// as if K2 had moved it.  resume: continue after the residual was replaced
// (partials from cg_rz_rr): x already holds this iteration's step, the stop
// tests are skipped.  Runs only when K2 completed this iteration (kk); block
// 0 records a stop in `done`, which K3 itself never reads.
template <typename T, bool ZMEM>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_update_xp(int32_t n, int32_t k_arg, int32_t g_rz, int32_t g_rr, int32_t resume, const T* __restrict__ r,
             const T* __restrict__ dinv, const T* __restrict__ z, T* __restrict__ x, T* __restrict__ p,
             const T* __restrict__ part, CgState<T>* st) {
#pragma clang fp contract(off)
    // iteration number: the argument, or the one K2 of this iteration wrote
    int32_t k = k_arg;
    if (!resume) {
        const int32_t kk = st->kk;
        if (kk < 0 || (k_arg >= 0 && kk != k_arg)) return;
        k = kk;
    }
    __shared__ T red[VEC_BLOCK / 64];
    const T rz = sum_partials_all<T, VEC_BLOCK>(part + PART_RZ, g_rz, red);
    const T rr = sum_partials_all<T, VEC_BLOCK>(part + PART_RR, g_rr, red);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    int32_t stop = CG_RUNNING;
    if (!resume && rr <= st->thresh) stop = CG_CONVERGED;
    else if (!(rz > T(0)) || !isfinite(rz)) stop = CG_BREAKDOWN;
    else if (!resume && rr <= st->pause_thresh) stop = CG_PAUSED;
    const T a = st->alpha;
    const int32_t i0 = blockIdx.x * VEC_BLOCK + threadIdx.x, di = gridDim.x * VEC_BLOCK;
    if (stop != CG_RUNNING) {
        if (!resume)
            for (int32_t i = i0; i < n; i += di) x[i] = x[i] + a * p[i];
        if (lead) {
            st->rr = rr;
            st->iter = k + 1;
            st->done = stop;
        }
        return;
    }
    const T beta = rz / st->rz[k & 3];
    // z = M^-1 r: Jacobi on the fly, or (ZMEM) as the block-Jacobi kernel
    // before this one stored it
    if (resume) {
        for (int32_t i = i0; i < n; i += di) p[i] = (ZMEM ? z[i] : dinv[i] * r[i]) + beta * p[i];
    } else {
        int32_t i = i0;
        constexpr int U = vec_unroll_xp<T>();
        for (; (int64_t)i + (int64_t)(U - 1) * di < n; i += U * di) {
            T zv[U], xv[U], pv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (ZMEM) {
                    zv[u] = z[i + u * di];
                } else {
                    const T ri = r[i + u * di];
                    zv[u] = dinv[i + u * di] * ri;
                }
                xv[u] = x[i + u * di];
                pv[u] = p[i + u * di];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                x[i + u * di] = xv[u] + a * pv[u];
                p[i + u * di] = zv[u] + beta * pv[u];
            }
        }
        for (; i < n; i += di) {
            const T pi = p[i];
            x[i] = x[i] + a * pi;
            p[i] = (ZMEM ? z[i] : dinv[i] * r[i]) + beta * pi;
        }
    }
    if (lead) {
        st->rz[(k + 1) & 3] = rz;
        st->rr = rr;
        st->beta = beta;
        st->iter = k + 1;
        if (resume) {
            st->rr_ref = rr;
            st->pause_thresh = st->pause_frac2 * rr;
            st->done = CG_RUNNING;
        }
    }
}

// K3 of iteration k fused with K1 of iteration k + 1 (systems of at most
// RP_LOOP_TWO_MAX_ROWS rows, Jacobi M, rows read as plain CSR).  The stop
// tests and x += alpha p_k are K3's.  Unless stopping, p_{k+1} = M^-1 r +
// beta p_k of a row is formed wherever it is needed: once by the row itself,
// which stores it into pn, and again, by the same operations, by every row
// coupled to it, so q = A p_{k+1} and the (p, q) partials come out of this
// launch.  p_k (po) and p_{k+1} (pn) are separate buffers; on a stop pn
// receives p_k, so after this kernel ran the current direction is in pn.
// Rows go to blocks as in K1 and each row sums its products in column order
// from 0, so q and the partials are K1's bit for bit.  Gated on kk like K3.
template <typename T>
__global__ void __launch_bounds__(SPMV_BLOCK)
cg_update_xp_spmv(int32_t n, int32_t k, int32_t g_vec, const int32_t* __restrict__ row_ptr,
                  const int32_t* __restrict__ col, const T* __restrict__ val, const T* __restrict__ r,
                  const T* __restrict__ dinv, const T* __restrict__ po, T* __restrict__ pn, T* __restrict__ x,
                  T* __restrict__ q, T* __restrict__ part, CgState<T>* st) {
#pragma clang fp contract(off)
    if (st->kk != k) return;
    __shared__ T red[SPMV_BLOCK / 64];
    const T rz = sum_partials_all<T, SPMV_BLOCK>(part + PART_RZ, g_vec, red);
    const T rr = sum_partials_all<T, SPMV_BLOCK>(part + PART_RR, g_vec, red);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    int32_t stop = CG_RUNNING;
    if (rr <= st->thresh) stop = CG_CONVERGED;
    else if (!(rz > T(0)) || !isfinite(rz)) stop = CG_BREAKDOWN;
    else if (rr <= st->pause_thresh) stop = CG_PAUSED;
    const T a = st->alpha;
    const int32_t n_groups = (int32_t)(((int64_t)n + SPMV_BLOCK - 1) / SPMV_BLOCK);
    const int32_t g0 = xcd_block(), gstep = (int32_t)gridDim.x;
    if (stop != CG_RUNNING) {
        for (int32_t g = g0; g < n_groups; g += gstep) {
            const int32_t i = g * SPMV_BLOCK + (int32_t)threadIdx.x;
            if (i < n) {
                const T pi = po[i];
                x[i] = x[i] + a * pi;
                pn[i] = pi;
            }
        }
        if (lead) {
            st->rr = rr;
            st->iter = k + 1;
            st->done = stop;
        }
        return;
    }
    const T beta = rz / st->rz[k & 3];
    const bool spmv = k + 1 < st->max_iter;   // K1 of iteration k + 1 runs
    T ppq = T(0);
    for (int32_t g = g0; g < n_groups; g += gstep) {
        const int32_t i = g * SPMV_BLOCK + (int32_t)threadIdx.x;
        if (i >= n) continue;
        const T pi = po[i];
        x[i] = x[i] + a * pi;
        const T pni = dinv[i] * r[i] + beta * pi;
        pn[i] = pni;
        if (spmv) {
            // U entries per trip, every load of a trip issued before its first
            // product; the products are added in column order as before
            constexpr int U = 8;
            T sum = T(0);
            const int32_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
            for (int32_t eb = e0; eb < e1; eb += U) {
                int32_t cj[U];
                T vv[U], rj[U], dj[U], pj[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool in = eb + u < e1;
                    cj[u] = in ? col[eb + u] : i;
                    vv[u] = in ? val[eb + u] : T(0);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    rj[u] = r[cj[u]];
                    dj[u] = dinv[cj[u]];
                    pj[u] = po[cj[u]];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (eb + u < e1) sum += vv[u] * (dj[u] * rj[u] + beta * pj[u]);
            }
            q[i] = sum;
            ppq += pni * sum;
        }
    }
    if (spmv) {
        const T b = block_sum<T, SPMV_BLOCK>(ppq, red);
        if (threadIdx.x == 0) part[PART_A + xcd_block()] = b;
    }
    if (lead) {
        st->rz[(k + 1) & 3] = rz;
        st->rr = rr;
        st->beta = beta;
        st->iter = k + 1;
    }
}

// x64 += (double) x32, then x32 = 0
__global__ void __launch_bounds__(VEC_BLOCK)
ir_accumulate(int32_t n, double* __restrict__ x, float* __restrict__ d) {
#pragma clang fp contract(off)
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        x[i] = x[i] + (double)d[i];
        d[i] = 0.0f;
    }
}

// ---------------------------------------------------------------------------
// block-Jacobi forms of the kernels that apply M^-1 (blocks of BS rows, one
// thread per block; packed inverses from precond.hip).  z_i sums over the
// block's j ascending, from 0, as the definition does.
// ---------------------------------------------------------------------------
template <int BS>
__device__ __forceinline__ constexpr int bj_idx(int i, int j) {
    return i <= j ? i * BS - i * (i - 1) / 2 + (j - i) : j * BS - j * (j - 1) / 2 + (i - j);
}

// zv[0..m) = M_b^-1 rv[0..m) for block b
template <typename T, int BS>
__device__ __forceinline__ void bj_block_solve(int32_t m, const T* __restrict__ mb, const T (&rv)[BS], T (&zv)[BS]) {
#pragma clang fp contract(off)
    constexpr int P = BS * (BS + 1) / 2;
    T pk[P];
#pragma unroll
    for (int q = 0; q < P; ++q) pk[q] = mb[q];
#pragma unroll
    for (int i = 0; i < BS; ++i) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < BS; ++j)
            if (j < m) s += pk[bj_idx<BS>(i, j)] * rv[j];
        zv[i] = s;
    }
}

// K2 with block-Jacobi: alpha = rz_k / (p, q); r -= alpha q; z = M^-1 r
// (stored for K3); partials of (r, z) -> PART_RZ and (r, r) -> PART_RR
template <typename T, int BS>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_update_r_bj(int32_t n, int32_t k_arg, int32_t g_spmv, int32_t nb, const int32_t* __restrict__ start,
               const T* __restrict__ minv, T* __restrict__ r, const T* __restrict__ q, T* __restrict__ z,
               T* __restrict__ part, CgState<T>* st) {
#pragma clang fp contract(off)
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (st->done != CG_RUNNING) {
        if (lead) st->kk = -1;
        return;
    }
    const int32_t k = k_arg >= 0 ? k_arg : st->iter;
    if (k >= st->max_iter) {
        if (lead) st->kk = -1;
        return;
    }
    __shared__ T red[VEC_BLOCK / 64];
    const T pq = sum_partials_all<T, VEC_BLOCK>(part + PART_A, g_spmv, red);
    if (!(pq > T(0)) || !isfinite(pq)) {
        if (lead) {
            st->pq = pq;
            st->iter = k;
            st->kk = -1;
            st->done = CG_BREAKDOWN;
        }
        return;
    }
    const T a = st->rz[k & 3] / pq;
    constexpr int P = BS * (BS + 1) / 2;
    T prz = T(0), prr = T(0);
    for (int32_t b = blockIdx.x * VEC_BLOCK + threadIdx.x; b < nb; b += gridDim.x * VEC_BLOCK) {
        const int32_t s0 = start[b], m = start[b + 1] - s0;
        T rv[BS], zv[BS];
#pragma unroll
        for (int j = 0; j < BS; ++j) {
            rv[j] = T(0);
            if (j < m) rv[j] = r[s0 + j] - a * q[s0 + j];
        }
        bj_block_solve<T, BS>(m, minv + (int64_t)b * P, rv, zv);
#pragma unroll
        for (int j = 0; j < BS; ++j)
            if (j < m) {
                r[s0 + j] = rv[j];
                z[s0 + j] = zv[j];
                prz += rv[j] * zv[j];
                prr += rv[j] * rv[j];
            }
    }
    const T b1 = block_sum<T, VEC_BLOCK>(prz, red);
    const T b2 = block_sum<T, VEC_BLOCK>(prr, red);
    if (threadIdx.x == 0) {
        part[PART_RZ + blockIdx.x] = b1;
        part[PART_RR + blockIdx.x] = b2;
    }
    if (lead) {
        st->pq = pq;
        st->alpha = a;
        st->kk = k;
    }
}

// start with block-Jacobi: p = M^-1 r; partials of (r, M^-1 r) -> PART_RZ.
// rz_rr: z = M^-1 r stored, partials of (r, z) -> PART_RZ and (r, r) -> PART_RR
template <typename T, int BS, bool RZ_RR>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_precond_bj(int32_t nb, const int32_t* __restrict__ start, const T* __restrict__ minv, const T* __restrict__ r,
              T* __restrict__ out, T* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ T red[VEC_BLOCK / 64];
    constexpr int P = BS * (BS + 1) / 2;
    T prz = T(0), prr = T(0);
    for (int32_t b = blockIdx.x * VEC_BLOCK + threadIdx.x; b < nb; b += gridDim.x * VEC_BLOCK) {
        const int32_t s0 = start[b], m = start[b + 1] - s0;
        T rv[BS], zv[BS];
#pragma unroll
        for (int j = 0; j < BS; ++j) rv[j] = j < m ? r[s0 + j] : T(0);
        bj_block_solve<T, BS>(m, minv + (int64_t)b * P, rv, zv);
#pragma unroll
        for (int j = 0; j < BS; ++j)
            if (j < m) {
                out[s0 + j] = zv[j];
                prz += rv[j] * zv[j];
                prr += rv[j] * rv[j];
            }
    }
    const T b1 = block_sum<T, VEC_BLOCK>(prz, red);
    if (RZ_RR) {
        const T b2 = block_sum<T, VEC_BLOCK>(prr, red);
        if (threadIdx.x == 0) part[PART_RR + blockIdx.x] = b2;
    }
    if (threadIdx.x == 0) part[PART_RZ + blockIdx.x] = b1;
}

// Lane-per-row forms for aligned blocks: every block starts at a multiple of
// BS (each rank's rows a multiple of BS) and BS divides 64, so a block's rows
// are BS neighbouring lanes of one wavefront.  Loads and stores are then
// coalesced like the Jacobi kernels'; a lane takes its block's residuals
// from its neighbours with shuffles and reads its own row of the packed
// inverse.  Same products and sums, in the same order, as the per-block
// form.
template <typename T, int BS>
__device__ __forceinline__ T bj_lane_solve(T ri, int32_t i, const T* __restrict__ minv) {
#pragma clang fp contract(off)
    constexpr int P = BS * (BS + 1) / 2;
    const int lane = threadIdx.x & 63;
    const int li = lane & (BS - 1);        // the row's place in its block
    const int l0 = lane - li;
    const T* mb = minv + (int64_t)(i / BS) * P;
    T mrow[BS];
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        const int a = li < j ? li : j, c = li < j ? j : li;
        mrow[j] = mb[a * BS - a * (a - 1) / 2 + (c - a)];
    }
    T zi = T(0);
#pragma unroll
    for (int j = 0; j < BS; ++j) zi += mrow[j] * __shfl(ri, l0 + j, 64);
    return zi;
}

template <typename T, int BS>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_update_r_bj_lane(int32_t n, int32_t k_arg, int32_t g_spmv, const T* __restrict__ minv, T* __restrict__ r,
                    const T* __restrict__ q, T* __restrict__ z, T* __restrict__ part, CgState<T>* st) {
#pragma clang fp contract(off)
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (st->done != CG_RUNNING) {
        if (lead) st->kk = -1;
        return;
    }
    const int32_t k = k_arg >= 0 ? k_arg : st->iter;
    if (k >= st->max_iter) {
        if (lead) st->kk = -1;
        return;
    }
    __shared__ T red[VEC_BLOCK / 64];
    const T pq = sum_partials_all<T, VEC_BLOCK>(part + PART_A, g_spmv, red);
    if (!(pq > T(0)) || !isfinite(pq)) {
        if (lead) {
            st->pq = pq;
            st->iter = k;
            st->kk = -1;
            st->done = CG_BREAKDOWN;
        }
        return;
    }
    const T a = st->rz[k & 3] / pq;
    T prz = T(0), prr = T(0);
    // whole wavefronts per trip (the grid stride is a multiple of 64), so a
    // block's lanes are active together; rows past n carry 0
    const int32_t di = gridDim.x * VEC_BLOCK;
    for (int32_t base = blockIdx.x * VEC_BLOCK; base < n; base += di) {
        const int32_t i = base + threadIdx.x;
        const bool in = i < n;
        const T ri = in ? r[i] - a * q[i] : T(0);
        const T zi = bj_lane_solve<T, BS>(ri, in ? i : 0, minv);
        if (in) {
            r[i] = ri;
            z[i] = zi;
            prz += ri * zi;
            prr += ri * ri;
        }
    }
    const T b1 = block_sum<T, VEC_BLOCK>(prz, red);
    const T b2 = block_sum<T, VEC_BLOCK>(prr, red);
    if (threadIdx.x == 0) {
        part[PART_RZ + blockIdx.x] = b1;
        part[PART_RR + blockIdx.x] = b2;
    }
    if (lead) {
        st->pq = pq;
        st->alpha = a;
        st->kk = k;
    }
}

template <typename T, int BS, bool RZ_RR>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_precond_bj_lane(int32_t n, const T* __restrict__ minv, const T* __restrict__ r, T* __restrict__ out,
                   T* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ T red[VEC_BLOCK / 64];
    T prz = T(0), prr = T(0);
    const int32_t di = gridDim.x * VEC_BLOCK;
    for (int32_t base = blockIdx.x * VEC_BLOCK; base < n; base += di) {
        const int32_t i = base + threadIdx.x;
        const bool in = i < n;
        const T ri = in ? r[i] : T(0);
        const T zi = bj_lane_solve<T, BS>(ri, in ? i : 0, minv);
        if (in) {
            out[i] = zi;
            prz += ri * zi;
            prr += ri * ri;
        }
    }
    const T b1 = block_sum<T, VEC_BLOCK>(prz, red);
    if (RZ_RR) {
        const T b2 = block_sum<T, VEC_BLOCK>(prr, red);
        if (threadIdx.x == 0) part[PART_RR + blockIdx.x] = b2;
    }
    if (threadIdx.x == 0) part[PART_RZ + blockIdx.x] = b1;
}

#define RP_DISPATCH_BS_LANE(bs, CALL) \
    do {                              \
        switch (bs) {                 \
        case 1: CALL(1); break;       \
        case 2: CALL(2); break;       \
        case 4: CALL(4); break;       \
        default: CALL(8); break;      \
        }                             \
    } while (0)

#define RP_DISPATCH_BS(bs, CALL) \
    do {                         \
        switch (bs) {            \
        case 1: CALL(1); break;  \
        case 2: CALL(2); break;  \
        case 3: CALL(3); break;  \
        case 4: CALL(4); break;  \
        case 5: CALL(5); break;  \
        case 6: CALL(6); break;  \
        case 7: CALL(7); break;  \
        default: CALL(8); break; \
        }                        \
    } while (0)

__global__ void fill_zero(int32_t n, double* x) {
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) x[i] = 0.0;
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
template <typename T>
struct Cg {
    rp_plan* plan;
    int32_t n;
    SpmvIdx ix;
    const T* val;
    const T* dinv;
    T* x;
    const T* b;
    T* r;
    T* p;
    T* q;
    T* part;
    CgState<T>* st;     // device
    CgState<T>* h;      // pinned host mirror
    int kernel_id;      // RP_KERNEL_SPMV64 / RP_KERNEL_SPMV32
    hipStream_t s;
    int32_t g_spmv, g_vec;
    int32_t xw_mode;
    XWin w;
    // block-Jacobi (bj_minv != nullptr): M^-1 by blocks; z holds M^-1 r for K3
    const int32_t* bj_start = nullptr;
    const T* bj_minv = nullptr;
    int32_t bj_nb = 0;
    int32_t bj_bs = 0;
    bool bj_lane = false;   // aligned blocks: the lane-per-row kernels
    T* z = nullptr;
    // multigrid (amg): M^-1 r = one V-cycle (amg.hip) into z; its last kernel
    // writes g_rz partials of (r, z), on the SpMV grid
    bool amg = false;
    bool amg_ordered = false;   // the hierarchy of the solve-order copy
    int32_t g_rz = 0;       // partials of (r, z) the finalize and K3 sum
    // two-launch iteration: the second direction buffer (p_k and p_{k+1}
    // alternate between p and p_alt; p always names the current one between
    // calls of iterate)
    T* p_alt = nullptr;
};

// the matrix a solve runs on: the fused pattern in the plan's SpMV form, or
// the solve-order copy (plain CSR groups, no x windows)
struct MatView {
    SpmvIdx ix;
    int32_t xw_mode;
};

MatView mat_view(rp_plan* p, bool ordered) {
    if (ordered) return MatView{SpmvIdx{p->d_ro_row_ptr, p->d_ro_col, nullptr, nullptr, nullptr}, -1};
    return MatView{spmv_idx(p), p->xw_mode};
}

template <typename T>
Cg<T> make_cg(rp_plan* p, const MatView& m, const T* val, const T* dinv, T* x, const T* b, T* r, T* pv, T* q,
              CgState<T>* st, CgState<T>* h, int kernel_id, hipStream_t s) {
    Cg<T> c{p, (int32_t)p->n_rows, m.ix, val, dinv, x, b, r, pv, q, (T*)p->d_partials, st, h,
            kernel_id, s, spmv_grid(p->n_rows), plan_vec_grid(p), m.xw_mode, XWin{{p->xw_d[0], p->xw_d[1]}}};
    c.g_rz = c.g_vec;
    return c;
}

template <typename T>
int read_state(Cg<T>& c) {
    RP_HIP_TRY(hipMemcpyAsync(c.h, c.st, sizeof(CgState<T>), hipMemcpyDeviceToHost, c.s));
    RP_HIP_TRY(hipStreamSynchronize(c.s));
    return RP_OK;
}

template <typename T, bool W32>
int launch_residual(Cg<T>& c, bool xzero, float* r32) {
    const dim3 g(c.g_spmv), bl(SPMV_BLOCK);
    if (xzero) {
        hipLaunchKernelGGL((residual_kernel<T, true, W32, -1>), g, bl, 0, c.s, c.n, c.ix, c.val, c.x,
                           c.b, c.r, r32, c.part, c.w);
    } else {
#define RP_LAUNCH(NW)                                                                                        \
    hipLaunchKernelGGL((residual_kernel<T, false, W32, NW>), g, bl, 0, c.s, c.n, c.ix, c.val, c.x, \
                       c.b, c.r, r32, c.part, c.w)
        RP_DISPATCH_NW(c.xw_mode, RP_LAUNCH);
#undef RP_LAUNCH
    }
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

template <typename T>
int launch_finalize(Cg<T>& c, int32_t mode, int32_t k, T tol2, T pause_frac2, int32_t max_iter = 0) {
    hipLaunchKernelGGL(cg_finalize<T>, dim3(1), dim3(VEC_BLOCK), 0, c.s, mode, k, max_iter, tol2, pause_frac2, c.g_spmv,
                       c.g_rz, c.part, c.st);
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

// (re)start at iteration k from the residual in r (the residual_kernel's
// partials are still in PART_A / PART_B)
template <typename T>
int launch_start(Cg<T>& c, int32_t k, T tol2, T pause_frac2, int32_t max_iter) {
    if (c.amg) {
        RP_TRY(amg_apply<T>(c.plan, c.r, c.p, c.part, c.g_rz, false, nullptr, c.s, c.amg_ordered));
    } else if (c.bj_minv && c.bj_lane) {
#define RP_LAUNCH(BS)                                                                                          \
    hipLaunchKernelGGL((cg_precond_bj_lane<T, BS, false>), dim3(c.g_vec), dim3(VEC_BLOCK), 0, c.s, c.n, c.bj_minv, \
                       c.r, c.p, c.part)
        RP_DISPATCH_BS_LANE(c.bj_bs, RP_LAUNCH);
#undef RP_LAUNCH
    } else if (c.bj_minv) {
#define RP_LAUNCH(BS)                                                                                          \
    hipLaunchKernelGGL((cg_precond_bj<T, BS, false>), dim3(c.g_vec), dim3(VEC_BLOCK), 0, c.s, c.bj_nb, c.bj_start, \
                       c.bj_minv, c.r, c.p, c.part)
        RP_DISPATCH_BS(c.bj_bs, RP_LAUNCH);
#undef RP_LAUNCH
    } else {
        hipLaunchKernelGGL(cg_start_p<T>, dim3(c.g_vec), dim3(VEC_BLOCK), 0, c.s, c.n, c.r, c.dinv, c.p, c.part);
    }
    RP_HIP_TRY(hipGetLastError());
    return launch_finalize(c, FIN_START, k, tol2, pause_frac2, max_iter);
}

// continue after r was replaced: beta from the new (r, z), p update, running again
template <typename T>
int launch_resume(Cg<T>& c) {
    const int32_t k = c.h->iter - 1;
    if (c.amg) {
        RP_TRY(amg_apply<T>(c.plan, c.r, c.z, c.part, c.g_rz, true, nullptr, c.s, c.amg_ordered));
        hipLaunchKernelGGL((cg_update_xp<T, true>), dim3(c.g_vec), dim3(VEC_BLOCK), 0, c.s, c.n, k, c.g_rz, c.g_rz, 1,
                           c.r, c.dinv, c.z, c.x, c.p, c.part, c.st);
    } else if (c.bj_minv) {
        if (c.bj_lane) {
#define RP_LAUNCH(BS)                                                                                         \
    hipLaunchKernelGGL((cg_precond_bj_lane<T, BS, true>), dim3(c.g_vec), dim3(VEC_BLOCK), 0, c.s, c.n, c.bj_minv, \
                       c.r, c.z, c.part)
            RP_DISPATCH_BS_LANE(c.bj_bs, RP_LAUNCH);
#undef RP_LAUNCH
        } else {
#define RP_LAUNCH(BS)                                                                                         \
    hipLaunchKernelGGL((cg_precond_bj<T, BS, true>), dim3(c.g_vec), dim3(VEC_BLOCK), 0, c.s, c.bj_nb, c.bj_start, \
                       c.bj_minv, c.r, c.z, c.part)
            RP_DISPATCH_BS(c.bj_bs, RP_LAUNCH);
#undef RP_LAUNCH
        }
        hipLaunchKernelGGL((cg_update_xp<T, true>), dim3(c.g_vec), dim3(VEC_BLOCK), 0, c.s, c.n, k, c.g_vec, c.g_vec, 1, c.r,
                           c.dinv, c.z, c.x, c.p, c.part, c.st);
    } else {
        hipLaunchKernelGGL(cg_rz_rr<T>, dim3(c.g_vec), dim3(VEC_BLOCK), 0, c.s, c.n, c.r, c.dinv, c.part);
        hipLaunchKernelGGL((cg_update_xp<T, false>), dim3(c.g_vec), dim3(VEC_BLOCK), 0, c.s, c.n, k, c.g_vec, c.g_vec, 1, c.r,
                           c.dinv, c.z, c.x, c.p, c.part, c.st);
    }
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

// one iteration as K1, K2, K3 on stream s (K1 between the timing events);
// k < 0: K2 and K3 take the iteration number from the device state (graphs)
template <typename T>
int launch_iteration(Cg<T>& c, int32_t k, hipStream_t s) {
    const dim3 gs(c.g_spmv), bs(SPMV_BLOCK), gv(c.g_vec), bv(VEC_BLOCK);
    RP_TRY(timing_begin(c.plan, c.kernel_id, s));
#define RP_LAUNCH(NW) \
    hipLaunchKernelGGL((cg_spmv_pq<T, NW>), gs, bs, 0, s, c.n, c.ix, c.val, c.p, c.q, c.part, c.st, c.w)
    RP_DISPATCH_NW(c.xw_mode, RP_LAUNCH);
#undef RP_LAUNCH
    RP_TRY(timing_end(c.plan, c.kernel_id, s));
    if (c.amg) {
        // K2 without (r, z); the V-cycle (skipped when K2 did no update)
        // stores z and the (r, z) partials; K3 reads z
        hipLaunchKernelGGL((cg_update_r<T, false>), gv, bv, 0, s, c.n, k, c.g_spmv, c.r, c.q, c.dinv, c.part, c.st);
        RP_HIP_TRY(hipGetLastError());
        RP_TRY(amg_apply<T>(c.plan, c.r, c.z, c.part, c.g_rz, false, &c.st->kk, s, c.amg_ordered));
        hipLaunchKernelGGL((cg_update_xp<T, true>), gv, bv, 0, s, c.n, k, c.g_rz, c.g_vec, 0, c.r, c.dinv, c.z, c.x,
                           c.p, c.part, c.st);
    } else if (c.bj_minv) {
        if (c.bj_lane) {
#define RP_LAUNCH(BS)                                                                                              \
    hipLaunchKernelGGL((cg_update_r_bj_lane<T, BS>), gv, bv, 0, s, c.n, k, c.g_spmv, c.bj_minv, c.r, c.q, c.z, c.part, \
                       c.st)
            RP_DISPATCH_BS_LANE(c.bj_bs, RP_LAUNCH);
#undef RP_LAUNCH
        } else {
#define RP_LAUNCH(BS)                                                                                          \
    hipLaunchKernelGGL((cg_update_r_bj<T, BS>), gv, bv, 0, s, c.n, k, c.g_spmv, c.bj_nb, c.bj_start, c.bj_minv, \
                       c.r, c.q, c.z, c.part, c.st)
            RP_DISPATCH_BS(c.bj_bs, RP_LAUNCH);
#undef RP_LAUNCH
        }
        hipLaunchKernelGGL((cg_update_xp<T, true>), gv, bv, 0, s, c.n, k, c.g_vec, c.g_vec, 0, c.r, c.dinv, c.z, c.x, c.p,
                           c.part, c.st);
    } else {
        hipLaunchKernelGGL(cg_update_r<T>, gv, bv, 0, s, c.n, k, c.g_spmv, c.r, c.q, c.dinv, c.part, c.st);
        hipLaunchKernelGGL((cg_update_xp<T, false>), gv, bv, 0, s, c.n, k, c.g_vec, c.g_vec, 0, c.r, c.dinv, c.z, c.x, c.p,
                           c.part, c.st);
    }
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

// The executable graph of `chunk` iterations for this Cg, captured on the
// plan's own stream and instantiated once; captured again when any kernel
// argument differs from the cached one's.
template <typename T>
int cg_graph(Cg<T>& c, int chunk, hipGraphExec_t* out) {
    rp_plan* p = c.plan;
    auto& g = p->cg_graph[sizeof(T) == 4 ? 1 : 0];
    const uint64_t key[24] = {(uint64_t)c.n,           (uint64_t)chunk,        (uint64_t)(uintptr_t)c.val,
                              (uint64_t)(uintptr_t)c.dinv, (uint64_t)(uintptr_t)c.x, (uint64_t)(uintptr_t)c.r,
                              (uint64_t)(uintptr_t)c.p,    (uint64_t)(uintptr_t)c.q, (uint64_t)(uintptr_t)c.part,
                              (uint64_t)(uintptr_t)c.st,   (uint64_t)(uintptr_t)c.ix.row_ptr,
                              (uint64_t)(uintptr_t)c.ix.col, (uint64_t)(uintptr_t)c.ix.goi_k,
                              (uint64_t)(uintptr_t)c.ix.goi_off, (uint64_t)(uintptr_t)c.ix.goi_mask,
                              (uint64_t)c.g_spmv,       (uint64_t)c.g_vec,      (uint64_t)(uint32_t)c.xw_mode,
                              (uint64_t)(uint32_t)c.w.d[0], (uint64_t)(uint32_t)c.w.d[1],
                              (uint64_t)(uintptr_t)c.bj_minv, (uint64_t)(uintptr_t)c.bj_start,
                              (uint64_t)(uintptr_t)c.z,
                              ((uint64_t)(uint32_t)c.bj_nb << 16) | ((uint32_t)c.bj_lane << 8) | (uint32_t)c.bj_bs};
    if (g.exec && std::memcmp(g.key, key, sizeof key) == 0) {
        *out = g.exec;
        return RP_OK;
    }
    if (g.exec) {
        RP_HIP_TRY(hipGraphExecDestroy(g.exec));
        g.exec = nullptr;
    }
    if (!p->capture_stream) RP_HIP_TRY(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = p->capture_stream;
    RP_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = RP_OK;
    for (int i = 0; i < chunk && rc == RP_OK; ++i) rc = launch_iteration(c, -1, cs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc != RP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    RP_HIP_TRY(e);
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    RP_HIP_TRY(ei);
    std::memcpy(g.key, key, sizeof key);
    *out = g.exec;
    return RP_OK;
}

// the plan's second direction buffer for the two-launch iteration: the
// preconditioned-residual vector, which Jacobi solves do not use otherwise
inline double* alt_direction(rp_plan* p, double*) { return p->d_z; }
inline float* alt_direction(rp_plan* p, float*) { return p->d_z32; }

// The two-launch form of the chunks below: K1 of the first iteration, then
// per iteration K2 and the fused K3 + K1 (cg_update_xp_spmv), until the
// state leaves CG_RUNNING or the budget is spent.  Same kernels' arithmetic,
// so the same iterates bit for bit.
template <typename T>
int iterate_two(Cg<T>& c, int chunk, int32_t max_iter) {
    RP_TRY(alloc_z(c.plan));
    if (!c.p_alt) c.p_alt = alt_direction(c.plan, c.p);
    T* pb[2] = {c.p, c.p_alt};
    const int32_t k0 = c.h->iter;
    const dim3 gs(c.g_spmv), bs(SPMV_BLOCK), gv(c.g_vec), bv(VEC_BLOCK);
#define RP_LAUNCH(NW) \
    hipLaunchKernelGGL((cg_spmv_pq<T, NW>), gs, bs, 0, c.s, c.n, c.ix, c.val, c.p, c.q, c.part, c.st, c.w)
    RP_DISPATCH_NW(c.xw_mode, RP_LAUNCH);
#undef RP_LAUNCH
    RP_HIP_TRY(hipGetLastError());
    while (c.h->done == CG_RUNNING && c.h->iter < max_iter) {
        const int32_t ks = c.h->iter;
        const int32_t k1 = (int32_t)std::min<int64_t>((int64_t)ks + chunk, max_iter);
        for (int32_t k = ks; k < k1; ++k) {
            hipLaunchKernelGGL(cg_update_r<T>, gv, bv, 0, c.s, c.n, k, c.g_spmv, c.r, c.q, c.dinv, c.part, c.st);
            hipLaunchKernelGGL(cg_update_xp_spmv<T>, gs, bs, 0, c.s, c.n, k, c.g_vec, c.ix.row_ptr, c.ix.col, c.val,
                               c.r, c.dinv, pb[(k - k0) & 1], pb[(k - k0 + 1) & 1], c.x, c.q, c.part, c.st);
        }
        RP_HIP_TRY(hipGetLastError());
        RP_TRY(read_state(c));
    }
    // The current direction: p_{iter} after a completed iteration, or p_k
    // after a stop in that kernel (it copied p_k forward), or p_k after a
    // breakdown in K2 of iteration k = iter (the fused kernel did not run).
    if ((c.h->iter - k0) & 1) std::swap(c.p, c.p_alt);
    return RP_OK;
}

// enqueue chunks of up to `chunk` iterations (never past max_iter) until the
// state leaves CG_RUNNING or the budget is spent.  graph: each chunk is one
// replay of a captured graph of `chunk` iterations (kernels past max_iter do
// nothing); per-kernel timing always launches eagerly.
template <typename T>
int iterate(Cg<T>& c, int chunk, int32_t max_iter, bool graph, int32_t fused_loop) {
    const bool timed = c.plan->timing.enabled;
    if (fused_loop == RP_LOOP_AUTO && c.n <= RP_LOOP_TWO_MAX_ROWS && !timed && !graph && !c.bj_minv && !c.amg)
        return iterate_two(c, chunk, max_iter);
    if (fused_loop == RP_LOOP_COOPERATIVE && !timed && !graph && !c.bj_minv && !c.amg) {
        // launches of at most LOOP_ITERS iterations keep the barrier counter
        // (3 arrivals per block and iteration) far below 2^32
        constexpr int64_t LOOP_ITERS = 1 << 16;
        bool ran = true;
        while (ran && c.h->done == CG_RUNNING && c.h->iter < max_iter) {
            const int32_t k1 = (int32_t)std::min<int64_t>((int64_t)c.h->iter + LOOP_ITERS, max_iter);
            RP_TRY(launch_cg_loop<T>(c.plan, c.n, c.ix, c.val, c.dinv, c.x, c.r, c.p, c.q, c.st, c.h->iter, k1, c.s,
                                     &ran));
            if (ran) RP_TRY(read_state(c));
        }
        if (ran) return RP_OK;
    }
    hipGraphExec_t exec = nullptr;
    if (graph && !timed && !c.amg) RP_TRY(cg_graph(c, chunk, &exec));
    while (c.h->done == CG_RUNNING && c.h->iter < max_iter) {
        const int32_t k0 = c.h->iter;
        if (exec) {
            RP_HIP_TRY(hipGraphLaunch(exec, c.s));
        } else {
            const int32_t k1 = (int32_t)std::min<int64_t>((int64_t)k0 + chunk, max_iter);
            for (int32_t k = k0; k < k1; ++k) RP_TRY(launch_iteration(c, k, c.s));
        }
        RP_TRY(read_state(c));
        if (!exec) RP_TRY(timing_collect(c.plan, c.kernel_id, (int64_t)c.h->iter - k0));
    }
    return RP_OK;
}

// block-Jacobi for this solve when the options ask for it
template <typename T>
void use_block_jacobi(Cg<T>& c, const rp_plan* p, const T* minv, T* z) {
    c.bj_start = p->d_bj_start;
    c.bj_minv = minv;
    c.bj_nb = (int32_t)p->bj_blocks;
    c.bj_bs = p->bj_bs;
    c.bj_lane = p->bj_aligned;
    c.z = z;
}

// the multigrid V-cycle for this solve (the hierarchy is current)
template <typename T>
void use_amg(Cg<T>& c, T* z, bool ordered) {
    c.amg = true;
    c.amg_ordered = ordered;
    c.z = z;
    c.g_rz = c.g_spmv;
}

int pending_value_error(rp_plan* p, hipStream_t s, bool need_symmetric) {
    RP_HIP_TRY(hipMemcpyAsync(p->h_flags, p->d_flags, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    if (p->h_flags[0] & FLAG_VALUE) {
        set_error("the last update produced a value that is not finite or a diagonal <= 0");
        return RP_ERR_VALUE;
    }
    if (need_symmetric && p->h_flags[1]) {
        set_error("CG needs a symmetric matrix: the last update has upper != lower or unequal "
                  "interface partners");
        return RP_ERR_UNSUPPORTED;
    }
    return RP_OK;
}

int check_solvable(rp_plan* p, hipStream_t s, bool need_symmetric = true) {
    if (!p->has_values) {
        set_error("rp_solve before any rp_update_values");
        return RP_ERR_ARG;
    }
    if (p->nnz_nl > 0) {
        set_error("the share has %lld non-local entries; the distributed solve is not part of this library",
                  (long long)p->nnz_nl);
        return RP_ERR_UNSUPPORTED;
    }
    return pending_value_error(p, s, need_symmetric);
}

}  // namespace

int values_solvable(rp_plan* p, hipStream_t s) { return check_solvable(p, s, true); }

int solve_fp64(rp_plan* p, const double* b, double* x, const rp_solve_opts& o, rp_solve_info& info,
               hipStream_t s, bool ordered) {
    RP_TRY(check_solvable(p, s));
    const MatView m = mat_view(p, ordered);
    Cg<double> c = make_cg<double>(p, m, ordered ? p->d_ro_val64 : p->d_val64,
                                   ordered ? p->d_ro_dinv64 : p->d_dinv64, x, b, p->d_r, p->d_p, p->d_q,
                                   p->d_st64, p->h_st64, RP_KERNEL_SPMV64, s);
    if (o.precond == RP_PRECOND_BLOCK_JACOBI) {
        RP_TRY(bj_prepare(p, o.block_size, s));
        use_block_jacobi(c, p, p->d_bj_minv64, p->d_z);
    } else if (o.precond == RP_PRECOND_AMG) {
        RP_TRY(amg_prepare(p, false, s, ordered));
        use_amg(c, p->d_z, ordered);
    }
    const double tol2 = o.tol * o.tol;
    const int chunk = std::max(1, o.check_every);
    RP_TRY((launch_residual<double, false>(c, o.x0_zero != 0, nullptr)));
    RP_TRY(launch_start(c, 0, tol2, 0.0, o.max_iter));
    RP_TRY(read_state(c));
    bool fresh = true;  // rr_true belongs to the current x
    int status = RP_NOT_CONVERGED;
    info.restarts = 0;
    for (;;) {
        const int32_t d = c.h->done;
        if (d == CG_ZERO_RHS) {
            hipLaunchKernelGGL(fill_zero, dim3(c.g_vec), dim3(VEC_BLOCK), 0, s, c.n, x);
            RP_HIP_TRY(hipGetLastError());
            status = RP_OK;
            break;
        }
        if (d == CG_CONVERGED) {
            if (!fresh) {
                RP_TRY((launch_residual<double, false>(c, false, nullptr)));
                RP_TRY(launch_finalize(c, FIN_RESIDUAL, 0, 0.0, 0.0));
                RP_TRY(read_state(c));
                fresh = true;
            }
            if (c.h->rr_true <= c.h->thresh) {
                status = RP_OK;
                break;
            }
            if (info.restarts >= o.max_restarts) break;
            ++info.restarts;
            RP_TRY(launch_start(c, c.h->iter, tol2, 0.0, o.max_iter));
            RP_TRY(read_state(c));
            continue;
        }
        if (d == CG_BREAKDOWN) {
            status = RP_ERR_BREAKDOWN;
            set_error("CG breakdown after %d iterations (p.Ap = %g)", c.h->iter, c.h->pq);
            break;
        }
        if (c.h->iter >= o.max_iter) break;
        RP_TRY(iterate(c, chunk, o.max_iter, o.graph != 0, o.fused_loop));
        fresh = false;
    }
    if (!fresh && c.h->done != CG_ZERO_RHS) {
        RP_TRY((launch_residual<double, false>(c, false, nullptr)));
        RP_TRY(launch_finalize(c, FIN_RESIDUAL, 0, 0.0, 0.0));
        RP_TRY(read_state(c));
    }
    info.iters = c.h->iter;
    info.outer_iters = 0;
    info.rel_res = c.h->bb > 0 ? std::sqrt(c.h->rr_true / c.h->bb) : 0.0;
    info.status = status;
    if (status == RP_NOT_CONVERGED)
        set_error("not converged: %d iterations, relative residual %g", info.iters, info.rel_res);
    return status;
}

int solve_mixed(rp_plan* p, const double* b, double* x, const rp_solve_opts& o, rp_solve_info& info,
                hipStream_t s, bool reliable, bool ordered) {
    RP_TRY(check_solvable(p, s));
    const MatView m = mat_view(p, ordered);
    // FP64: r64 = b - A x and its norm; x is the FP64 solution
    Cg<double> out = make_cg<double>(p, m, ordered ? p->d_ro_val64 : p->d_val64,
                                     ordered ? p->d_ro_dinv64 : p->d_dinv64, x, b, p->d_r, p->d_p, p->d_q,
                                     p->d_st_outer, p->h_st_outer, RP_KERNEL_SPMV64, s);
    // FP32 PCG on A32 d = r32 (b and r alias r32); d is folded into x
    Cg<float> in = make_cg<float>(p, m, ordered ? p->d_ro_val32 : p->d_val32,
                                  ordered ? p->d_ro_dinv32 : p->d_dinv32, p->d_x32, p->d_r32, p->d_r32, p->d_p32,
                                  p->d_q32, p->d_st32, p->h_st32, RP_KERNEL_SPMV32, s);
    if (o.precond == RP_PRECOND_BLOCK_JACOBI) {
        RP_TRY(bj_prepare(p, o.block_size, s));
        use_block_jacobi(in, p, p->d_bj_minv32, p->d_z32);
    } else if (o.precond == RP_PRECOND_AMG) {
        RP_TRY(amg_prepare(p, true, s, ordered));
        use_amg(in, p->d_z32, ordered);
    }
    const int chunk = std::max(1, o.check_every);

    RP_TRY((launch_residual<double, true>(out, o.x0_zero != 0, p->d_r32)));
    RP_TRY(launch_finalize(out, FIN_RESIDUAL, 0, 0.0, 0.0));
    RP_TRY(read_state(out));
    const double bb = out.h->bb;
    const double thresh = o.tol * o.tol * bb;
    double rr = out.h->rr_true;
    int status = RP_NOT_CONVERGED;
    int32_t outer = 0, total_inner = 0, stall = 0;
    if (bb == 0.0) {
        hipLaunchKernelGGL(fill_zero, dim3(out.g_vec), dim3(VEC_BLOCK), 0, s, out.n, x);
        RP_HIP_TRY(hipGetLastError());
        rr = 0.0;
        status = RP_OK;
    } else if (rr <= thresh) {
        status = RP_OK;
    }

    // FP32 PCG from d = 0 on the current r32 (the start clears x32).
    // reliable: never stops on its own; pauses after each update_delta
    // reduction of its residual.  Otherwise: stops once its residual is below
    // inner_tol times its start, or below half the outer target tol ||b||
    // (whichever comes first): a last refinement step need not go further
    // than the solve asks for.
    const float pause2 = reliable ? (float)(o.update_delta * o.update_delta) : 0.0f;
    bool start_inner = true;
    while (status != RP_OK) {
        if (start_inner) {
            float tol2_in = 0.0f;
            if (!reliable) {
                const double floor2 = 0.25 * thresh / rr;   // (tol ||b|| / 2)^2 relative to ||r||^2
                tol2_in = (float)std::min(0.25, std::max(o.inner_tol * o.inner_tol, floor2));
            }
            RP_TRY((launch_residual<float, false>(in, true, nullptr)));
            RP_TRY(launch_start(in, total_inner, tol2_in, pause2, o.max_iter));
            RP_TRY(read_state(in));
            start_inner = false;
        }
        const int32_t it_before = in.h->iter;
        RP_TRY(iterate(in, chunk, o.max_iter, o.graph != 0, o.fused_loop));
        total_inner = in.h->iter;
        const int32_t d = in.h->done;
        // fold the FP32 correction into x and take the FP64 residual
        hipLaunchKernelGGL(ir_accumulate, dim3(out.g_vec), dim3(VEC_BLOCK), 0, s, out.n, x, p->d_x32);
        RP_HIP_TRY(hipGetLastError());
        RP_TRY((launch_residual<double, true>(out, false, p->d_r32)));
        RP_TRY(launch_finalize(out, FIN_RESIDUAL, 0, 0.0, 0.0));
        RP_TRY(read_state(out));
        ++outer;
        const double rr_new = out.h->rr_true;
        if (rr_new <= thresh) {
            rr = rr_new;
            status = RP_OK;
            break;
        }
        stall = (rr_new > 0.25 * rr) ? stall + 1 : 0;
        rr = rr_new;
        if (d == CG_BREAKDOWN && in.h->iter == it_before) {
            status = RP_ERR_BREAKDOWN;
            set_error("FP32 CG breakdown (p.Ap = %g)", (double)in.h->pq);
            break;
        }
        if (total_inner >= o.max_iter || outer >= o.max_outer || stall >= 4) break;
        if (reliable && d == CG_PAUSED) {
            RP_TRY(launch_resume(in));   // keep the search direction, replaced residual
            RP_TRY(read_state(in));
        } else {
            start_inner = true;          // restart FP32 PCG on the new residual
        }
    }
    info.iters = total_inner;
    info.outer_iters = outer;
    info.restarts = 0;
    info.rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    info.status = status;
    if (status == RP_NOT_CONVERGED)
        set_error("mixed solve not converged: %d FP64 updates, %d FP32 iterations, relative residual %g",
                  outer, total_inner, info.rel_res);
    return status;
}


// ---------------------------------------------------------------------------
// BiCGStab (non-symmetric systems; the momentum solver of Sec. 4)
// ---------------------------------------------------------------------------
// Jacobi right-preconditioned BiCGStab (van der Vorst 1992), iteration k as
// five kernels; every kernel re-sums the previous kernel's partials, as in CG:
//   A  stop test on (r, r); rho = (rh, r); beta = (rho / rho_{k-1})(alpha / omega);
//      p = r + beta (p - omega v); y = M^-1 p
//   B  v = A y                        partials of (rh, v)
//   C  alpha = rho / (rh, v); s = r - alpha v; z = M^-1 s;   partials of (s, s)
//   D  stop at the half step if (s, s) is small; t = A z;    partials of (t, s), (t, t)
//   E  omega = (t, s) / (t, t); x = (x + alpha y) + omega z; r = s - omega t;
//      partials of (rh, r) and (r, r)
// A half-step stop in D of iteration k leaves done = BI_HALF and half_k = k;
// E of iteration k then moves x by alpha y, and the solve ends there (BI_HALF
// counts as converged).  E never writes `done` on that path, so its blocks
// all see the same BI_HALF whatever their order.
namespace {

// rh = r, p = v = 0; partials of (rh, r) -> PART_RZ and (r, r) -> PART_RR;
// rho_{k-1} = alpha = omega = 1 for the first iteration k
__global__ void __launch_bounds__(VEC_BLOCK)
bi_start(int32_t n, int32_t k, const double* __restrict__ r, double* __restrict__ rh, double* __restrict__ p,
         double* __restrict__ v, double* __restrict__ part, BiState* st) {
#pragma clang fp contract(off)
    __shared__ double red[VEC_BLOCK / 64];
    double prr = 0.0;
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        const double ri = r[i];
        rh[i] = ri;
        p[i] = 0.0;
        v[i] = 0.0;
        prr += ri * ri;
    }
    const double b = block_sum<double, VEC_BLOCK>(prr, red);
    if (threadIdx.x == 0) {
        part[PART_RZ + blockIdx.x] = b;
        part[PART_RR + blockIdx.x] = b;
        if (blockIdx.x == 0) {
            st->rho[(k + 3) & 3] = 1.0;
            st->alpha = 1.0;
            st->omega = 1.0;
        }
    }
}

// one block: rr_true and bb from residual_kernel's partials; with `start`
// also the convergence threshold and the state of a (re)started iteration k
__global__ void __launch_bounds__(VEC_BLOCK)
bi_finalize(int32_t start, int32_t k, double tol2, int32_t g_spmv, const double* __restrict__ part, BiState* st) {
#pragma clang fp contract(off)
    __shared__ double red[VEC_BLOCK / 64];
    const double rr = sum_partials_all<double, VEC_BLOCK>(part + PART_A, g_spmv, red);
    const double bb = sum_partials_all<double, VEC_BLOCK>(part + PART_B, g_spmv, red);
    if (threadIdx.x != 0) return;
    st->rr_true = rr;
    st->bb = bb;
    if (!start) return;
    const double thresh = tol2 * bb;
    st->thresh = thresh;
    st->rr = rr;
    st->iter = k;
    int32_t d = CG_RUNNING;
    if (bb == 0.0) d = CG_ZERO_RHS;
    else if (rr <= thresh) d = CG_CONVERGED;
    st->done = d;
}

// A
__global__ void __launch_bounds__(VEC_BLOCK)
bi_direction(int32_t n, int32_t k, int32_t g_vec, const double* __restrict__ r, const double* __restrict__ dinv,
             double* __restrict__ p, const double* __restrict__ v, double* __restrict__ y,
             const double* __restrict__ part, BiState* st) {
#pragma clang fp contract(off)
    if (st->done != CG_RUNNING) return;
    __shared__ double red[VEC_BLOCK / 64];
    const double rho = sum_partials_all<double, VEC_BLOCK>(part + PART_RZ, g_vec, red);
    const double rr = sum_partials_all<double, VEC_BLOCK>(part + PART_RR, g_vec, red);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const double omega = st->omega;
    int32_t stop = CG_RUNNING;
    if (rr <= st->thresh) stop = CG_CONVERGED;
    else if (rho == 0.0 || !isfinite(rho) || omega == 0.0) stop = CG_BREAKDOWN;
    if (stop != CG_RUNNING) {
        if (lead) {
            st->rr = rr;
            st->iter = k;
            st->done = stop;
        }
        return;
    }
    const double beta = (rho / st->rho[(k + 3) & 3]) * (st->alpha / omega);
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        const double pi = r[i] + beta * (p[i] - omega * v[i]);
        p[i] = pi;
        y[i] = dinv[i] * pi;
    }
    if (lead) {
        st->rho[k & 3] = rho;
        st->rr = rr;
    }
}

// B: v = A y; partials of (rh, v) -> PART_A
template <int NW>
__global__ void __launch_bounds__(SPMV_BLOCK)
bi_spmv_rv(int32_t n, SpmvIdx ix, const double* __restrict__ val, const double* __restrict__ y,
           double* __restrict__ v, const double* __restrict__ rh, double* __restrict__ part, const BiState* st,
           XWin w) {
#pragma clang fp contract(off)
    if (st->done != CG_RUNNING) return;
    __shared__ __align__(16) double lds[SPMV_CAP];
    __shared__ double xs[XWinSize<NW>::value];
    __shared__ double red[SPMV_BLOCK / 64];
    double prv = 0.0;
    GroupRange gr = block_groups(ix, n);
    for (int32_t g = gr.g0; g < gr.n_groups; g += gr.step) {
        const int32_t r0 = g * SPMV_BLOCK;
        const int32_t nr = min(SPMV_BLOCK, n - r0);
        const GroupRow<double> gr_ = spmv_group_row<double, NW>(ix, val, y, n, g, nr, w, xs, lds, gr);
        if ((int32_t)threadIdx.x < nr) {
            const int32_t i = r0 + threadIdx.x;
            v[i] = gr_.s;
            prv += rh[i] * gr_.s;
        }
    }
    const double b = block_sum<double, SPMV_BLOCK>(prv, red);
    if (threadIdx.x == 0) part[PART_A + xcd_block()] = b;
}

// C: alpha = rho / (rh, v); s = r - alpha v; z = M^-1 s; partials of (s, s) -> PART_RR
__global__ void __launch_bounds__(VEC_BLOCK)
bi_half(int32_t n, int32_t k, int32_t g_spmv, const double* __restrict__ r, const double* __restrict__ v,
        const double* __restrict__ dinv, double* __restrict__ s, double* __restrict__ z, double* __restrict__ part,
        BiState* st) {
#pragma clang fp contract(off)
    if (st->done != CG_RUNNING) return;
    __shared__ double red[VEC_BLOCK / 64];
    const double rv = sum_partials_all<double, VEC_BLOCK>(part + PART_A, g_spmv, red);
    if (rv == 0.0 || !isfinite(rv)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->iter = k;
            st->done = CG_BREAKDOWN;
        }
        return;
    }
    const double a = st->rho[k & 3] / rv;
    double pss = 0.0;
    // top down (e = n - 1 - i), like bi_update: the SpMVs and bi_direction
    // sweep bottom up, so each kernel starts on its predecessor's most recent
    // lines (still in the memory-side cache)
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        const int32_t e = n - 1 - i;
        const double si = r[e] - a * v[e];
        s[e] = si;
        z[e] = dinv[e] * si;
        pss += si * si;
    }
    const double b = block_sum<double, VEC_BLOCK>(pss, red);
    if (threadIdx.x == 0) {
        part[PART_RR + blockIdx.x] = b;
        if (blockIdx.x == 0) st->alpha = a;
    }
}

// D: half-step stop test on (s, s); t = A z; partials of (t, s) -> PART_A, (t, t) -> PART_B
template <int NW>
__global__ void __launch_bounds__(SPMV_BLOCK)
bi_spmv_ts(int32_t n, int32_t k, int32_t g_vec, SpmvIdx ix, const double* __restrict__ val,
           const double* __restrict__ z, double* __restrict__ t, const double* __restrict__ s,
           double* __restrict__ part, BiState* st, XWin w) {
#pragma clang fp contract(off)
    if (st->done != CG_RUNNING) return;
    __shared__ __align__(16) double lds[SPMV_CAP];
    __shared__ double xs[XWinSize<NW>::value];
    __shared__ double red[SPMV_BLOCK / 64];
    const double ss = sum_partials_all<double, VEC_BLOCK>(part + PART_RR, g_vec, red);
    if (ss <= st->thresh) {
        if (xcd_block() == 0 && threadIdx.x == 0) {
            st->rr = ss;
            st->half_k = k;
            st->done = BI_HALF;
        }
        return;
    }
    double pts = 0.0, ptt = 0.0;
    GroupRange gr = block_groups(ix, n);
    for (int32_t g = gr.g0; g < gr.n_groups; g += gr.step) {
        const int32_t r0 = g * SPMV_BLOCK;
        const int32_t nr = min(SPMV_BLOCK, n - r0);
        const GroupRow<double> gr_ = spmv_group_row<double, NW>(ix, val, z, n, g, nr, w, xs, lds, gr);
        if ((int32_t)threadIdx.x < nr) {
            const int32_t i = r0 + threadIdx.x;
            t[i] = gr_.s;
            pts += gr_.s * s[i];
            ptt += gr_.s * gr_.s;
        }
    }
    const double b1 = block_sum<double, SPMV_BLOCK>(pts, red);
    const double b2 = block_sum<double, SPMV_BLOCK>(ptt, red);
    if (threadIdx.x == 0) {
        part[PART_A + xcd_block()] = b1;
        part[PART_B + xcd_block()] = b2;
    }
}

// E: omega = (t, s) / (t, t); x = (x + alpha y) + omega z; r = s - omega t;
// partials of (rh, r) -> PART_RZ and (r, r) -> PART_RR.  After a half-step
// stop in this iteration's D (half_k == k): x += alpha y only.
__global__ void __launch_bounds__(VEC_BLOCK)
bi_update(int32_t n, int32_t k, int32_t g_spmv, double* __restrict__ x, const double* __restrict__ y,
          const double* __restrict__ z, const double* __restrict__ s, const double* __restrict__ t,
          const double* __restrict__ rh, double* __restrict__ r, double* __restrict__ part, BiState* st) {
#pragma clang fp contract(off)
    const int32_t d = st->done;
    if (d != CG_RUNNING && d != BI_HALF) return;
    __shared__ double red[VEC_BLOCK / 64];
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const double a = st->alpha;
    const int32_t i0 = blockIdx.x * VEC_BLOCK + threadIdx.x, di = gridDim.x * VEC_BLOCK;
    if (d == BI_HALF) {
        if (st->half_k != k) return;
        for (int32_t i = i0; i < n; i += di) x[i] = x[i] + a * y[i];
        if (lead) st->iter = k + 1;
        return;
    }
    const double ts = sum_partials_all<double, VEC_BLOCK>(part + PART_A, g_spmv, red);
    const double tt = sum_partials_all<double, VEC_BLOCK>(part + PART_B, g_spmv, red);
    if (tt == 0.0 || !isfinite(tt)) {
        if (lead) {
            st->iter = k + 1;
            st->done = CG_BREAKDOWN;
        }
        return;
    }
    const double omega = ts / tt;
    double prho = 0.0, prr = 0.0;
    for (int32_t i = i0; i < n; i += di) {  // top down, see bi_half
        const int32_t e = n - 1 - i;
        const double xi = (x[e] + a * y[e]) + omega * z[e];
        const double ri = s[e] - omega * t[e];
        x[e] = xi;
        r[e] = ri;
        prho += rh[e] * ri;
        prr += ri * ri;
    }
    const double b1 = block_sum<double, VEC_BLOCK>(prho, red);
    const double b2 = block_sum<double, VEC_BLOCK>(prr, red);
    if (threadIdx.x == 0) {
        part[PART_RZ + blockIdx.x] = b1;
        part[PART_RR + blockIdx.x] = b2;
        if (blockIdx.x == 0) {
            st->omega = omega;
            st->iter = k + 1;
        }
    }
}

struct Bi {
    Cg<double> c;   // matrix, x, b, r, partials; its CgState holds residual norms
    double *rh, *p, *v, *y, *s, *z, *t;
    BiState* st;
    BiState* h;
};

int bi_read(Bi& q) {
    RP_HIP_TRY(hipMemcpyAsync(q.h, q.st, sizeof(BiState), hipMemcpyDeviceToHost, q.c.s));
    RP_HIP_TRY(hipStreamSynchronize(q.c.s));
    return RP_OK;
}

// r = b - A x (x cleared first when xzero) and a (re)start at iteration k
int bi_launch_start(Bi& q, bool xzero, int32_t k, double tol2) {
    Cg<double>& c = q.c;
    RP_TRY((launch_residual<double, false>(c, xzero, nullptr)));
    hipLaunchKernelGGL(bi_start, dim3(c.g_vec), dim3(VEC_BLOCK), 0, c.s, c.n, k, c.r, q.rh, q.p, q.v, c.part,
                       q.st);
    hipLaunchKernelGGL(bi_finalize, dim3(1), dim3(VEC_BLOCK), 0, c.s, 1, k, tol2, c.g_spmv, c.part, q.st);
    RP_HIP_TRY(hipGetLastError());
    return bi_read(q);
}

// rr_true of the current x (r is overwritten)
int bi_true_residual(Bi& q) {
    Cg<double>& c = q.c;
    RP_TRY((launch_residual<double, false>(c, false, nullptr)));
    hipLaunchKernelGGL(bi_finalize, dim3(1), dim3(VEC_BLOCK), 0, c.s, 0, 0, 0.0, c.g_spmv, c.part, q.st);
    RP_HIP_TRY(hipGetLastError());
    return bi_read(q);
}

int bi_iterate(Bi& q, int chunk, int32_t max_iter) {
    Cg<double>& c = q.c;
    const dim3 gs(c.g_spmv), bs(SPMV_BLOCK), gv(c.g_vec), bv(VEC_BLOCK);
    while (q.h->done == CG_RUNNING && q.h->iter < max_iter) {
        const int32_t k0 = q.h->iter;
        const int32_t k1 = (int32_t)std::min<int64_t>((int64_t)k0 + chunk, max_iter);
        for (int32_t k = k0; k < k1; ++k) {
            hipLaunchKernelGGL(bi_direction, gv, bv, 0, c.s, c.n, k, c.g_vec, c.r, c.dinv, q.p, q.v, q.y, c.part,
                               q.st);
#define RP_LAUNCH(NW)                                                                                        \
    hipLaunchKernelGGL((bi_spmv_rv<NW>), gs, bs, 0, c.s, c.n, c.ix, c.val, q.y, q.v, q.rh, c.part, q.st, c.w)
            RP_DISPATCH_NW(c.xw_mode, RP_LAUNCH);
#undef RP_LAUNCH
            hipLaunchKernelGGL(bi_half, gv, bv, 0, c.s, c.n, k, c.g_spmv, c.r, q.v, c.dinv, q.s, q.z, c.part, q.st);
#define RP_LAUNCH(NW)                                                                                         \
    hipLaunchKernelGGL((bi_spmv_ts<NW>), gs, bs, 0, c.s, c.n, k, c.g_vec, c.ix, c.val, q.z, q.t, q.s, c.part, \
                       q.st, c.w)
            RP_DISPATCH_NW(c.xw_mode, RP_LAUNCH);
#undef RP_LAUNCH
            hipLaunchKernelGGL(bi_update, gv, bv, 0, c.s, c.n, k, c.g_spmv, c.x, q.y, q.z, q.s, q.t, q.rh, c.r,
                               c.part, q.st);
        }
        RP_HIP_TRY(hipGetLastError());
        RP_TRY(bi_read(q));
    }
    return RP_OK;
}

}  // namespace

int solve_bicgstab(rp_plan* p, const double* b, double* x, const rp_solve_opts& o, rp_solve_info& info,
                   hipStream_t s, bool ordered) {
    RP_TRY(check_solvable(p, s, false));
    const int64_t n = p->n_rows;
    if (!p->d_bi_work) RP_HIP_TRY(hipMalloc(&p->d_bi_work, sizeof(double) * 5 * (size_t)n));
    // A^T x = b: same pattern and diagonal, transposed values (the solve-order
    // copy of them is gathered by the caller)
    if (o.transpose && !ordered) RP_TRY(build_transpose(p, s));
    const double* val = ordered ? (o.transpose ? p->d_ro_valT : p->d_ro_val64)
                                : (o.transpose ? p->d_valT : p->d_val64);
    Bi q{make_cg<double>(p, mat_view(p, ordered), val, ordered ? p->d_ro_dinv64 : p->d_dinv64, x, b, p->d_r,
                         p->d_p, p->d_q, p->d_st64, p->h_st64, RP_KERNEL_SPMV64, s),
         p->d_bi_work, p->d_p, p->d_q, p->d_bi_work + n, p->d_bi_work + 2 * n, p->d_bi_work + 3 * n,
         p->d_bi_work + 4 * n, p->d_bi_st, p->h_bi_st};
    const double tol2 = o.tol * o.tol;
    const int chunk = std::max(1, o.check_every);
    RP_TRY(bi_launch_start(q, o.x0_zero != 0, 0, tol2));
    bool fresh = true;  // rr_true belongs to the current x
    int status = RP_NOT_CONVERGED;
    info.restarts = 0;
    for (;;) {
        const int32_t d = q.h->done;
        if (d == CG_ZERO_RHS) {
            hipLaunchKernelGGL(fill_zero, dim3(q.c.g_vec), dim3(VEC_BLOCK), 0, s, q.c.n, x);
            RP_HIP_TRY(hipGetLastError());
            status = RP_OK;
            break;
        }
        if (d == CG_CONVERGED || d == BI_HALF) {
            if (!fresh) {
                RP_TRY(bi_true_residual(q));
                fresh = true;
            }
            if (q.h->rr_true <= q.h->thresh) {
                status = RP_OK;
                break;
            }
            if (info.restarts >= o.max_restarts) break;
            ++info.restarts;
            RP_TRY(bi_launch_start(q, false, q.h->iter, tol2));
            continue;
        }
        if (d == CG_BREAKDOWN) {
            status = RP_ERR_BREAKDOWN;
            set_error("BiCGStab breakdown after %d iterations", q.h->iter);
            break;
        }
        if (q.h->iter >= o.max_iter) break;
        RP_TRY(bi_iterate(q, chunk, o.max_iter));
        fresh = false;
    }
    if (!fresh && q.h->done != CG_ZERO_RHS) RP_TRY(bi_true_residual(q));
    info.iters = q.h->iter;
    info.outer_iters = 0;
    info.rel_res = q.h->bb > 0 ? std::sqrt(q.h->rr_true / q.h->bb) : 0.0;
    info.status = status;
    if (status == RP_NOT_CONVERGED)
        set_error("not converged: %d iterations, relative residual %g", info.iters, info.rel_res);
    return status;
}

}  // namespace rp

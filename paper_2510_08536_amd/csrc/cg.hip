// Jacobi-preconditioned CG (the CG pressure solve of Sec. 4, M = diag(A)) and
// the FP32-inner / FP64-outer iterative refinement built on it.
//
// One iteration is three kernels; all scalars stay on the device:
//   K1  q = A p, pq = (p, q)                   -> alpha = rz / pq
//   K2  x += alpha p, r -= alpha q, z = M^-1 r,
//       rz' = (r, z), rr = (r, r)              -> stop test, beta = rz'/rz
//   K3  p = M^-1 r + beta p
// Each reduction ends in the block that arrives last, which sums the
// per-block partials in index order (deterministic, no floating-point
// atomics) and updates the state.  Once the state says "done", every later
// kernel returns at entry, so the host can enqueue iterations in chunks and
// read the state only between chunks; the iteration count does not depend on
// the chunk length.  The stop test is ||r||^2 <= tol^2 ||b||^2 on the
// recurrence residual, then confirmed on b - A x; a failed confirmation
// restarts CG from the current x.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "spmv.hpp"

namespace rp {

namespace {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// r = b - A x (x = 0 when XZERO, and then x is cleared), partial sums of
// (r, r) and (b, b); with W32 also r32 = RNE(r).  Last block stores rr_true
// and bb.
template <typename T, bool XZERO, bool W32>
__global__ void __launch_bounds__(SPMV_BLOCK)
residual_kernel(int32_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                const T* __restrict__ val, T* __restrict__ x, const T* b, T* r, float* r32,
                T* __restrict__ part, CgState<T>* st) {
#pragma clang fp contract(off)
    __shared__ T lds[XZERO ? 1 : SPMV_CAP];
    __shared__ T red[SPMV_BLOCK / 64];
    T prr = T(0), pbb = T(0);
    const GroupRange gr = block_groups(n);
    for (int32_t g = gr.g0; g < gr.g1; ++g) {
        const int32_t r0 = g * SPMV_BLOCK;
        const int32_t nr = min(SPMV_BLOCK, n - r0);
        T s = T(0);
        if (!XZERO) s = spmv_group_row(row_ptr, col, val, x, r0, nr, lds);
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
    const int32_t L = xcd_block();
    if (threadIdx.x == 0) {
        store_partial(part + L, brr);
        store_partial(part + MAX_PARTIALS + L, bbb);
    }
    if (arrive_last(&st->counter[0], gridDim.x)) {
        const T rr = sum_partials<T, SPMV_BLOCK>(part, gridDim.x, red);
        const T bb = sum_partials<T, SPMV_BLOCK>(part + MAX_PARTIALS, gridDim.x, red);
        if (threadIdx.x == 0) {
            st->rr_true = rr;
            st->bb = bb;
            st->counter[0] = 0;
        }
    }
}

// start (or restart) CG from the residual in r: p = M^-1 r, rz = (r, p)
template <typename T>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_start(int32_t n, const T* __restrict__ r, const T* __restrict__ dinv, T* __restrict__ p, T tol2,
         T* __restrict__ part, CgState<T>* st) {
#pragma clang fp contract(off)
    __shared__ T red[VEC_BLOCK / 64];
    T prz = T(0);
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        const T ri = r[i];
        const T zi = dinv[i] * ri;
        p[i] = zi;
        prz += ri * zi;
    }
    const T brz = block_sum<T, VEC_BLOCK>(prz, red);
    if (threadIdx.x == 0) store_partial(part + blockIdx.x, brz);
    if (arrive_last(&st->counter[0], gridDim.x)) {
        const T rz = sum_partials<T, VEC_BLOCK>(part, gridDim.x, red);
        if (threadIdx.x == 0) {
            const T thresh = tol2 * st->bb;
            st->rz = rz;
            st->rr = st->rr_true;
            st->thresh = thresh;
            int32_t d = CG_RUNNING;
            if (st->bb == T(0)) d = CG_ZERO_RHS;
            else if (st->rr_true <= thresh) d = CG_CONVERGED;
            else if (!(rz > T(0)) || !isfinite(rz)) d = CG_BREAKDOWN;
            else if (st->iter >= st->max_iter) d = CG_MAX_ITER;
            st->done = d;
            st->counter[0] = 0;
        }
    }
}

// K1: q = A p, pq = (p, q), alpha = rz / pq
template <typename T>
__global__ void __launch_bounds__(SPMV_BLOCK)
cg_spmv_pq(int32_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
           const T* __restrict__ val, const T* __restrict__ p, T* __restrict__ q, T* __restrict__ part,
           CgState<T>* st) {
#pragma clang fp contract(off)
    if (st->done != CG_RUNNING) return;
    __shared__ T lds[SPMV_CAP];
    __shared__ T red[SPMV_BLOCK / 64];
    T ppq = T(0);
    const GroupRange gr = block_groups(n);
    for (int32_t g = gr.g0; g < gr.g1; ++g) {
        const int32_t r0 = g * SPMV_BLOCK;
        const int32_t nr = min(SPMV_BLOCK, n - r0);
        const T s = spmv_group_row(row_ptr, col, val, p, r0, nr, lds);
        if ((int32_t)threadIdx.x < nr) {
            const int32_t i = r0 + threadIdx.x;
            q[i] = s;
            ppq += p[i] * s;
        }
    }
    const T bpq = block_sum<T, SPMV_BLOCK>(ppq, red);
    if (threadIdx.x == 0) store_partial(part + xcd_block(), bpq);
    if (arrive_last(&st->counter[0], gridDim.x)) {
        const T pq = sum_partials<T, SPMV_BLOCK>(part, gridDim.x, red);
        if (threadIdx.x == 0) {
            st->pq = pq;
            if (!(pq > T(0)) || !isfinite(pq)) st->done = CG_BREAKDOWN;
            else st->alpha = st->rz / pq;
            st->counter[0] = 0;
        }
    }
}

// K2: x += alpha p, r -= alpha q, rz' = (r, M^-1 r), rr = (r, r); stop test, beta
template <typename T>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_update_xr(int32_t n, T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
             const T* __restrict__ q, const T* __restrict__ dinv, T* __restrict__ part, CgState<T>* st) {
#pragma clang fp contract(off)
    if (st->done != CG_RUNNING) return;
    __shared__ T red[VEC_BLOCK / 64];
    const T a = st->alpha;
    T prz = T(0), prr = T(0);
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        const T xi = x[i] + a * p[i];
        const T ri = r[i] - a * q[i];
        x[i] = xi;
        r[i] = ri;
        const T zi = dinv[i] * ri;
        prz += ri * zi;
        prr += ri * ri;
    }
    const T brz = block_sum<T, VEC_BLOCK>(prz, red);
    const T brr = block_sum<T, VEC_BLOCK>(prr, red);
    if (threadIdx.x == 0) {
        store_partial(part + blockIdx.x, brz);
        store_partial(part + MAX_PARTIALS + blockIdx.x, brr);
    }
    if (arrive_last(&st->counter[1], gridDim.x)) {
        const T rz = sum_partials<T, VEC_BLOCK>(part, gridDim.x, red);
        const T rr = sum_partials<T, VEC_BLOCK>(part + MAX_PARTIALS, gridDim.x, red);
        if (threadIdx.x == 0) {
            const int32_t it = st->iter + 1;
            st->iter = it;
            st->rr = rr;
            if (rr <= st->thresh) st->done = CG_CONVERGED;
            else if (!(rz > T(0)) || !isfinite(rz)) st->done = CG_BREAKDOWN;
            else if (it >= st->max_iter) st->done = CG_MAX_ITER;
            else {
                st->beta = rz / st->rz;
                st->rz = rz;
            }
            st->counter[1] = 0;
        }
    }
}

// K3: p = M^-1 r + beta p
template <typename T>
__global__ void __launch_bounds__(VEC_BLOCK)
cg_update_p(int32_t n, const T* __restrict__ r, const T* __restrict__ dinv, T* __restrict__ p,
            const CgState<T>* st) {
#pragma clang fp contract(off)
    if (st->done != CG_RUNNING) return;
    const T beta = st->beta;
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK)
        p[i] = dinv[i] * r[i] + beta * p[i];
}

// refinement: x += (double) d
__global__ void __launch_bounds__(VEC_BLOCK)
ir_accumulate(int32_t n, double* __restrict__ x, const float* __restrict__ d) {
#pragma clang fp contract(off)
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK)
        x[i] = x[i] + (double)d[i];
}

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
    const int32_t* row_ptr;
    const int32_t* col;
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
};

template <typename T>
int read_state(Cg<T>& c) {
    RP_HIP_TRY(hipMemcpyAsync(c.h, c.st, sizeof(CgState<T>), hipMemcpyDeviceToHost, c.s));
    RP_HIP_TRY(hipStreamSynchronize(c.s));
    return RP_OK;
}

template <typename T>
int init_state(Cg<T>& c, int32_t max_iter) {
    CgState<T> z;
    std::memset(&z, 0, sizeof(z));
    z.max_iter = max_iter;
    z.done = CG_RUNNING;
    // the pinned mirror is the copy source; make sure an earlier read is done
    RP_HIP_TRY(hipStreamSynchronize(c.s));
    *c.h = z;
    RP_HIP_TRY(hipMemcpyAsync(c.st, c.h, sizeof(CgState<T>), hipMemcpyHostToDevice, c.s));
    return RP_OK;
}

template <typename T, bool W32>
int launch_residual(Cg<T>& c, bool xzero, float* r32) {
    const dim3 g(spmv_grid(c.n)), bl(SPMV_BLOCK);
    if (xzero)
        hipLaunchKernelGGL((residual_kernel<T, true, W32>), g, bl, 0, c.s, c.n, c.row_ptr, c.col, c.val, c.x,
                           c.b, c.r, r32, c.part, c.st);
    else
        hipLaunchKernelGGL((residual_kernel<T, false, W32>), g, bl, 0, c.s, c.n, c.row_ptr, c.col, c.val, c.x,
                           c.b, c.r, r32, c.part, c.st);
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

template <typename T>
int launch_start(Cg<T>& c, T tol2) {
    hipLaunchKernelGGL(cg_start<T>, dim3(vec_grid(c.n)), dim3(VEC_BLOCK), 0, c.s, c.n, c.r, c.dinv, c.p, tol2,
                       c.part, c.st);
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

// enqueue chunks of `chunk` iterations until the state leaves CG_RUNNING
template <typename T>
int iterate(Cg<T>& c, int chunk) {
    const dim3 gs(spmv_grid(c.n)), bs(SPMV_BLOCK), gv(vec_grid(c.n)), bv(VEC_BLOCK);
    while (c.h->done == CG_RUNNING) {
        const int32_t it0 = c.h->iter;
        for (int k = 0; k < chunk; ++k) {
            RP_TRY(timing_begin(c.plan, c.kernel_id, c.s));
            hipLaunchKernelGGL(cg_spmv_pq<T>, gs, bs, 0, c.s, c.n, c.row_ptr, c.col, c.val, c.p, c.q, c.part,
                               c.st);
            RP_TRY(timing_end(c.plan, c.kernel_id, c.s));
            hipLaunchKernelGGL(cg_update_xr<T>, gv, bv, 0, c.s, c.n, c.x, c.r, c.p, c.q, c.dinv, c.part, c.st);
            hipLaunchKernelGGL(cg_update_p<T>, gv, bv, 0, c.s, c.n, c.r, c.dinv, c.p, c.st);
        }
        RP_HIP_TRY(hipGetLastError());
        RP_TRY(read_state(c));
        RP_TRY(timing_collect(c.plan, c.kernel_id, (int64_t)c.h->iter - it0));
    }
    return RP_OK;
}

int pending_value_error(rp_plan* p, hipStream_t s) {
    RP_HIP_TRY(hipMemcpyAsync(p->h_flags, p->d_flags, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    if (p->h_flags[0] & FLAG_VALUE) {
        set_error("the last update produced a value that is not finite or a diagonal <= 0");
        return RP_ERR_VALUE;
    }
    if (p->h_flags[1]) {
        set_error("CG needs a symmetric matrix: the last update has upper != lower or unequal "
                  "interface partners");
        return RP_ERR_UNSUPPORTED;
    }
    return RP_OK;
}

int check_solvable(rp_plan* p, hipStream_t s) {
    if (!p->has_values) {
        set_error("rp_solve before any rp_update_values");
        return RP_ERR_ARG;
    }
    if (p->nnz_nl > 0) {
        set_error("the share has %lld non-local entries; the distributed solve is not part of this library",
                  (long long)p->nnz_nl);
        return RP_ERR_UNSUPPORTED;
    }
    return pending_value_error(p, s);
}

}  // namespace

int solve_fp64(rp_plan* p, const double* b, double* x, const rp_solve_opts& o, rp_solve_info& info,
               hipStream_t s) {
    RP_TRY(check_solvable(p, s));
    Cg<double> c{p, (int32_t)p->n_rows, p->d_row_ptr, p->d_col, p->d_val64, p->d_dinv64, x, b,
                 p->d_r, p->d_p, p->d_q, (double*)p->d_partials, p->d_st64, p->h_st64,
                 RP_KERNEL_SPMV64, s};
    const double tol2 = o.tol * o.tol;
    const int chunk = std::max(1, o.check_every);
    RP_TRY(init_state(c, o.max_iter));
    RP_TRY((launch_residual<double, false>(c, o.x0_zero != 0, nullptr)));
    RP_TRY(launch_start(c, tol2));
    RP_TRY(read_state(c));
    bool fresh = true;  // rr_true belongs to the current x
    int status = RP_NOT_CONVERGED;
    info.restarts = 0;
    for (;;) {
        const int32_t d = c.h->done;
        if (d == CG_ZERO_RHS) {
            hipLaunchKernelGGL(fill_zero, dim3(vec_grid(c.n)), dim3(VEC_BLOCK), 0, s, c.n, x);
            RP_HIP_TRY(hipGetLastError());
            status = RP_OK;
            break;
        }
        if (d == CG_CONVERGED) {
            if (!fresh) {
                RP_TRY((launch_residual<double, false>(c, false, nullptr)));
                RP_TRY(read_state(c));
                fresh = true;
            }
            if (c.h->rr_true <= c.h->thresh) {
                status = RP_OK;
                break;
            }
            if (info.restarts >= o.max_restarts) break;
            ++info.restarts;
            RP_TRY(launch_start(c, tol2));
            RP_TRY(read_state(c));
            continue;
        }
        if (d == CG_BREAKDOWN) {
            status = RP_ERR_BREAKDOWN;
            set_error("CG breakdown after %d iterations (p.Ap = %g)", c.h->iter, c.h->pq);
            break;
        }
        if (d == CG_MAX_ITER) break;
        RP_TRY(iterate(c, chunk));
        fresh = false;
    }
    if (!fresh && c.h->done != CG_ZERO_RHS) {
        RP_TRY((launch_residual<double, false>(c, false, nullptr)));
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
                hipStream_t s) {
    RP_TRY(check_solvable(p, s));
    const int32_t n = (int32_t)p->n_rows;
    // outer FP64 residual: r64 = b - A x, r32 = RNE(r64)
    Cg<double> out{p, n, p->d_row_ptr, p->d_col, p->d_val64, p->d_dinv64, x, b, p->d_r, p->d_p, p->d_q,
                   (double*)p->d_partials, p->d_st_outer, p->h_st64, RP_KERNEL_SPMV64, s};
    // inner FP32 PCG on A32 d = r32 from d = 0 (b and r alias r32)
    Cg<float> in{p, n, p->d_row_ptr, p->d_col, p->d_val32, p->d_dinv32, p->d_x32, p->d_r32, p->d_r32,
                 p->d_p32, p->d_q32, (float*)p->d_partials, p->d_st32, p->h_st32, RP_KERNEL_SPMV32, s};
    const int chunk = std::max(1, o.check_every);
    const float itol2 = (float)(o.inner_tol * o.inner_tol);

    RP_TRY(init_state(out, 0));
    RP_TRY((launch_residual<double, true>(out, o.x0_zero != 0, p->d_r32)));
    RP_TRY(read_state(out));
    const double bb = out.h->bb;
    const double thresh = o.tol * o.tol * bb;
    int status = RP_NOT_CONVERGED;
    int32_t total_inner = 0, outer = 0, stall = 0;
    double rr = out.h->rr_true;
    if (bb == 0.0) {
        hipLaunchKernelGGL(fill_zero, dim3(vec_grid(n)), dim3(VEC_BLOCK), 0, s, n, x);
        RP_HIP_TRY(hipGetLastError());
        status = RP_OK;
        rr = 0.0;
    } else if (rr <= thresh) {
        status = RP_OK;
    }
    while (status != RP_OK && outer < o.max_outer && total_inner < o.max_iter) {
        ++outer;
        RP_TRY(init_state(in, o.max_iter - total_inner));
        RP_TRY((launch_residual<float, false>(in, true, nullptr)));
        RP_TRY(launch_start(in, itol2));
        RP_TRY(read_state(in));
        RP_TRY(iterate(in, chunk));
        total_inner += in.h->iter;
        hipLaunchKernelGGL(ir_accumulate, dim3(vec_grid(n)), dim3(VEC_BLOCK), 0, s, n, x, p->d_x32);
        RP_HIP_TRY(hipGetLastError());
        RP_TRY((launch_residual<double, true>(out, false, p->d_r32)));
        RP_TRY(read_state(out));
        const double rr_new = out.h->rr_true;
        if (rr_new <= thresh) {
            rr = rr_new;
            status = RP_OK;
            break;
        }
        // no progress from the FP32 correction for three steps: give up
        stall = (rr_new > 0.25 * rr) ? stall + 1 : 0;
        rr = rr_new;
        if (stall >= 3 || in.h->iter == 0) break;
    }
    info.iters = total_inner;
    info.outer_iters = outer;
    info.restarts = 0;
    info.rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    info.status = status;
    if (status == RP_NOT_CONVERGED)
        set_error("mixed refinement not converged: %d outer, %d inner iterations, relative residual %g", outer,
                  total_inner, info.rel_res);
    return status;
}

}  // namespace rp

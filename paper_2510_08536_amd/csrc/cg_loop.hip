// CG iterations in one cooperative launch (rp_solve_opts.fused_loop).
//
// On small systems an iteration is bound by the gaps between its three
// dependent kernels, not by memory.  Here one launch, with every block
// resident at once (cooperative launch), runs the iterations itself: the
// three phases of an iteration (q = A p with (p, q); r -= alpha q with
// (r, M^-1 r) and (r, r); x and p updates with the stop tests) are separated
// by grid-wide barriers instead of kernel boundaries.  The arithmetic, the
// per-block partial sums and the device state are those of the three-kernel
// iteration in cg.hip (each phase re-sums the previous phase's partials in
// index order, every block the same scalars); every block takes every stop
// decision from the same sums, so all leave the loop together.
//
// The barrier: each block has a flag word of its own (one 128-byte line per
// block).  Arriving, the block's first thread publishes the block's writes
// (agent-scope release fence) and stores the barrier's sequence number into
// the block's flag; the first wave then polls every block's flag until all
// hold that number and takes an agent-scope acquire fence.  One release and
// one acquire per block and barrier: on this device they write back and
// invalidate the die's L2, so their count, not the polling, sets the cost of
// a barrier, and a grid of few blocks (several row groups per block) keeps it
// low.  The wait is bounded: after BAR_SPINS polls the block sets the abort
// word and leaves, and every block that sees the abort word leaves too; the
// host reports it.  The flags and the abort word are cleared by a kernel
// before each launch.
#include "spmv.hpp"

namespace rp {

namespace {

constexpr uint32_t BAR_SPINS = 1u << 22;   // a few seconds of polling at most
constexpr int FLAG_STRIDE = 32;            // words: one 128-byte line per block flag
constexpr int FLAG0 = FLAG_STRIDE;         // word 0: abort word; flags from line 1
constexpr int LOOP_GRID_MAX = 128;

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// all blocks of the grid; false when the wait was abandoned.  seq counts
// the barriers of this launch (the same in every block).
__device__ __forceinline__ bool grid_barrier(uint32_t* bar, uint32_t& seq) {
    __shared__ uint32_t ok;
    ++seq;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(bar + FLAG0 + FLAG_STRIDE * blockIdx.x, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x < 64) {
        uint32_t good = 1, spins = 0;
        for (;;) {
            int pending = 0;
            for (int b = threadIdx.x; b < (int)gridDim.x; b += 64)
                pending |= load_relaxed(bar + FLAG0 + FLAG_STRIDE * b) < seq;
            if (!__any(pending)) break;
            // the abort word and the count are the same in every lane
            if (load_relaxed(bar) != 0u || ++spins > BAR_SPINS) {
                if (threadIdx.x == 0) atomicOr(bar, 1u);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (threadIdx.x == 0) ok = good;
    }
    __syncthreads();
    return ok != 0;
}

__global__ void clear_barrier(uint32_t* bar, int32_t words) {
    for (int32_t i = threadIdx.x; i < words; i += blockDim.x) bar[i] = 0u;
}

template <typename T>
__global__ void __launch_bounds__(SPMV_BLOCK)
cg_loop(int32_t n, SpmvIdx ix, const T* __restrict__ val, const T* __restrict__ dinv, T* x, T* r, T* p, T* q,
        T* part, CgState<T>* st, int32_t k0, int32_t k_end, uint32_t* bar) {
    // x, r, p, q and the partials are written by other blocks between
    // barriers: no __restrict__ on them
#pragma clang fp contract(off)
    __shared__ __align__(16) T lds[SPMV_CAP];
    __shared__ T xs[1];
    __shared__ T red[SPMV_BLOCK / 64];
    if (st->done != CG_RUNNING) return;
    const XWin w{{0, 0}};
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const int32_t G = gridDim.x;
    const int32_t i0 = blockIdx.x * SPMV_BLOCK + threadIdx.x, di = G * SPMV_BLOCK;
    const int32_t k_stop = min(k_end, st->max_iter);
    uint32_t seq = 0;
    for (int32_t k = k0; k < k_stop; ++k) {
        // q = A p, partials of (p, q)
        T ppq = T(0);
        GroupRange gr = block_groups(ix, n);
        for (int32_t g = gr.g0; g < gr.n_groups; g += gr.step) {
            const int32_t r0 = g * SPMV_BLOCK;
            const int32_t nr = min(SPMV_BLOCK, n - r0);
            const GroupRow<T> row = spmv_group_row<T, -1>(ix, val, p, n, g, nr, w, xs, lds, gr);
            if ((int32_t)threadIdx.x < nr) {
                const int32_t i = r0 + threadIdx.x;
                q[i] = row.s;
                ppq += own_x<T, -1>(i, row, xs, p) * row.s;
            }
        }
        const T bpq = block_sum<T, SPMV_BLOCK>(ppq, red);
        if (threadIdx.x == 0) part[PART_A + xcd_block()] = bpq;
        if (!grid_barrier(bar, seq)) return;

        // alpha = rz_k / (p, q); r -= alpha q; partials of (r, M^-1 r), (r, r)
        const T pq = sum_partials_all<T, SPMV_BLOCK>(part + PART_A, G, red);
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
        for (int32_t i = i0; i < n; i += di) {
            const T ri = r[i] - a * q[i];
            r[i] = ri;
            prz += ri * (dinv[i] * ri);
            prr += ri * ri;
        }
        const T b1 = block_sum<T, SPMV_BLOCK>(prz, red);
        const T b2 = block_sum<T, SPMV_BLOCK>(prr, red);
        if (threadIdx.x == 0) {
            part[PART_RZ + blockIdx.x] = b1;
            part[PART_RR + blockIdx.x] = b2;
        }
        if (!grid_barrier(bar, seq)) return;

        // x += alpha p; stop tests; beta = rz_{k+1} / rz_k; p = M^-1 r + beta p
        const T rz = sum_partials_all<T, SPMV_BLOCK>(part + PART_RZ, G, red);
        const T rr = sum_partials_all<T, SPMV_BLOCK>(part + PART_RR, G, red);
        int32_t stop = CG_RUNNING;
        if (rr <= st->thresh) stop = CG_CONVERGED;
        else if (!(rz > T(0)) || !isfinite(rz)) stop = CG_BREAKDOWN;
        else if (rr <= st->pause_thresh) stop = CG_PAUSED;
        if (stop != CG_RUNNING) {
            for (int32_t i = i0; i < n; i += di) x[i] = x[i] + a * p[i];
            if (lead) {
                st->pq = pq;
                st->alpha = a;
                st->rr = rr;
                st->iter = k + 1;
                st->done = stop;
            }
            return;
        }
        const T beta = rz / st->rz[k & 3];
        for (int32_t i = i0; i < n; i += di) {
            const T pi = p[i];
            x[i] = x[i] + a * pi;
            p[i] = dinv[i] * r[i] + beta * pi;
        }
        if (lead) {
            st->rz[(k + 1) & 3] = rz;
            st->pq = pq;
            st->alpha = a;
            st->rr = rr;
            st->beta = beta;
            st->iter = k + 1;
        }
        if (!grid_barrier(bar, seq)) return;
    }
}

// blocks of the cooperative launch for n rows: about two groups of rows per
// block, at most LOOP_GRID_MAX blocks (a barrier costs about one L2
// write-back and invalidate per block, so fewer, fuller blocks are cheaper
// up to the point where the SpMV phase lacks parallelism), a multiple of 8,
// at most what the device holds at once
constexpr int BAR_WORDS = FLAG0 + FLAG_STRIDE * SPMV_GRID_MAX;

template <typename T>
int loop_grid(int64_t n, int* out) {
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    RP_HIP_TRY(hipGetDevice(&dev));
    RP_HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) {
        *out = 0;
        return RP_OK;
    }
    RP_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    RP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, cg_loop<T>, SPMV_BLOCK, 0));
    int64_t cap = std::min<int64_t>((int64_t)cus * per_cu, SPMV_GRID_MAX);
    cap -= cap % N_XCD;
    const int64_t groups = (n + SPMV_BLOCK - 1) / SPMV_BLOCK;
    int64_t g = std::min<int64_t>((groups + 1) / 2, LOOP_GRID_MAX);
    g = ((g + N_XCD - 1) / N_XCD) * N_XCD;
    *out = (int)std::max<int64_t>(std::min(g, cap), 0);
    return RP_OK;
}

}  // namespace

template <typename T>
int launch_cg_loop(rp_plan* p, int32_t n, const SpmvIdx& ix, const T* val, const T* dinv, T* x, T* r, T* pv, T* q,
                   CgState<T>* st, int32_t k0, int32_t k_end, hipStream_t s, bool* ran) {
    *ran = false;
    int grid = 0;
    RP_TRY(loop_grid<T>(n, &grid));
    if (grid < N_XCD) return RP_OK;
    if (!p->d_loop_bar) RP_HIP_TRY(hipMalloc(&p->d_loop_bar, BAR_WORDS * sizeof(uint32_t)));
    hipLaunchKernelGGL(clear_barrier, dim3(1), dim3(1024), 0, s, p->d_loop_bar, FLAG0 + FLAG_STRIDE * grid);
    RP_HIP_TRY(hipGetLastError());
    T* part = (T*)p->d_partials;
    uint32_t* bar = p->d_loop_bar;
    void* args[] = {&n, (void*)&ix, (void*)&val, (void*)&dinv, &x, &r, &pv, &q, &part, &st, &k0, &k_end, &bar};
    RP_HIP_TRY(hipLaunchCooperativeKernel((const void*)cg_loop<T>, dim3(grid), dim3(SPMV_BLOCK), args, 0, s));
    uint32_t abort_word = 0;
    RP_HIP_TRY(hipMemcpyAsync(&abort_word, p->d_loop_bar, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    if (abort_word) {
        set_error("the single-launch CG loop gave up waiting at a grid barrier");
        return RP_ERR_HIP;
    }
    *ran = true;
    return RP_OK;
}

template int launch_cg_loop<double>(rp_plan*, int32_t, const SpmvIdx&, const double*, const double*, double*,
                                    double*, double*, double*, CgState<double>*, int32_t, int32_t, hipStream_t, bool*);
template int launch_cg_loop<float>(rp_plan*, int32_t, const SpmvIdx&, const float*, const float*, float*, float*,
                                   float*, float*, CgState<float>*, int32_t, int32_t, hipStream_t, bool*);

}  // namespace rp

// extern "C" entry points of librp (declared in include/rp.h): argument
// checks, allocation, stream plumbing and error reporting around the
// kernels.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>

#include "rp_internal.hpp"

namespace rp {

namespace {
thread_local char g_err[1024] = "";
}

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

int timing_begin(rp_plan* p, int kernel, hipStream_t s) {
    if (!p->timing.enabled) return RP_OK;
    EventPool& e = p->timing.pool[kernel];
    const int64_t k = e.seen++;
    e.open = k % p->timing.stride == 0;
    if (!e.open) return RP_OK;
    if (e.used == (int64_t)e.start.size()) {
        hipEvent_t a, b;
        RP_HIP_TRY(hipEventCreate(&a));
        RP_HIP_TRY(hipEventCreate(&b));
        e.start.push_back(a);
        e.stop.push_back(b);
        e.idx.push_back(0);
    }
    e.idx[e.used] = k - e.chunk0;
    RP_HIP_TRY(hipEventRecord(e.start[e.used], s));
    return RP_OK;
}

int timing_end(rp_plan* p, int kernel, hipStream_t s) {
    if (!p->timing.enabled) return RP_OK;
    EventPool& e = p->timing.pool[kernel];
    if (!e.open) return RP_OK;
    RP_HIP_TRY(hipEventRecord(e.stop[e.used], s));
    ++e.used;
    e.open = false;
    return RP_OK;
}

// adds the recorded launches among the first `keep` launches since the last
// collection (the rest found the solve stopped) to the kernel's totals
int timing_collect(rp_plan* p, int kernel, int64_t keep) {
    EventPool& e = p->timing.pool[kernel];
    if (!p->timing.enabled || e.used == 0) {
        e.used = 0;
        e.chunk0 = e.seen;
        return RP_OK;
    }
    for (int64_t i = 0; i < e.used; ++i) {
        if (e.idx[i] >= keep) continue;
        float ms = 0.f;
        RP_HIP_TRY(hipEventSynchronize(e.stop[i]));
        RP_HIP_TRY(hipEventElapsedTime(&ms, e.start[i], e.stop[i]));
        p->timing.launches[kernel] += 1;
        p->timing.total_ms[kernel] += ms;
    }
    e.used = 0;
    e.chunk0 = e.seen;
    return RP_OK;
}

namespace {

void free_plan(rp_plan* p) {
    if (!p) return;
    void* dev[] = {p->d_slot_off, p->d_row0, p->d_nf, p->d_face_off, p->d_owner, p->d_nbr, p->d_iface_off,
                   p->d_row_ptr, p->d_col, p->d_perm, p->d_perm_inv, p->d_nl_row_ptr, p->d_nl_col, p->d_iface_partner, p->d_recv,
                   p->d_val64, p->d_val32, p->d_dinv64, p->d_dinv32, p->d_r, p->d_p, p->d_q, p->d_r32,
                   p->d_p32, p->d_q32, p->d_x32, p->d_partials, p->d_st64, p->d_st32, p->d_st_outer,
                   p->d_flags, p->d_goi_k, p->d_goi_off, p->d_goi_mask, p->d_bi_st, p->d_bi_work,
                   p->d_valT, p->d_tflag, p->d_ro_perm, p->d_ro_row_ptr, p->d_ro_col, p->d_ro_sig,
                   p->d_ro_val64, p->d_ro_val32, p->d_ro_dinv64, p->d_ro_dinv32, p->d_ro_b, p->d_ro_x,
                   p->d_ro_valT, (void*)p->d_src, p->d_bj_start, p->d_bj_minv64, p->d_bj_minv32, p->d_z,
                   p->d_z32, p->d_bj_flag, p->d_loop_bar};
    amg_free(p);
    for (void* q : dev)
        if (q) (void)hipFree(q);
    if (p->h_st64) (void)hipHostFree(p->h_st64);
    if (p->h_st32) (void)hipHostFree(p->h_st32);
    if (p->h_st_outer) (void)hipHostFree(p->h_st_outer);
    if (p->h_bi_st) (void)hipHostFree(p->h_bi_st);
    if (p->h_flags) (void)hipHostFree(p->h_flags);
    for (auto& g : p->cg_graph)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    for (auto& e : p->timing.pool) {
        for (hipEvent_t ev : e.start) (void)hipEventDestroy(ev);
        for (hipEvent_t ev : e.stop) (void)hipEventDestroy(ev);
    }
    delete p;
}

template <typename T>
int dalloc(T** q, int64_t count) {
    RP_HIP_TRY(hipMalloc(q, sizeof(T) * (size_t)std::max<int64_t>(count, 1)));
    return RP_OK;
}

int alloc_values(rp_plan* p) {
    const int64_t n = p->n_rows, ns = p->n_slots;
    RP_TRY(dalloc(&p->d_recv, ns));
    // SpMV pack loads may touch SPMV_PAD elements past the values
    RP_TRY(dalloc(&p->d_val64, ns + SPMV_PAD));
    RP_TRY(dalloc(&p->d_val32, ns + SPMV_PAD));
    RP_HIP_TRY(hipMemset(p->d_val64 + ns, 0, sizeof(double) * SPMV_PAD));
    RP_HIP_TRY(hipMemset(p->d_val32 + ns, 0, sizeof(float) * SPMV_PAD));
    RP_TRY(dalloc(&p->d_dinv64, n));
    RP_TRY(dalloc(&p->d_dinv32, n));
    RP_TRY(dalloc(&p->d_r, n));
    RP_TRY(dalloc(&p->d_p, n));
    RP_TRY(dalloc(&p->d_q, n));
    RP_TRY(dalloc(&p->d_r32, n));
    RP_TRY(dalloc(&p->d_p32, n));
    RP_TRY(dalloc(&p->d_q32, n));
    RP_TRY(dalloc(&p->d_x32, n));
    RP_HIP_TRY(hipMalloc(&p->d_partials, sizeof(double) * PART_TOTAL));
    RP_TRY(dalloc(&p->d_st64, 1));
    RP_TRY(dalloc(&p->d_st32, 1));
    RP_TRY(dalloc(&p->d_st_outer, 1));
    RP_HIP_TRY(hipMemset(p->d_st64, 0, sizeof(CgState<double>)));
    RP_HIP_TRY(hipMemset(p->d_st32, 0, sizeof(CgState<float>)));
    RP_HIP_TRY(hipMemset(p->d_st_outer, 0, sizeof(CgState<double>)));
    RP_HIP_TRY(hipHostMalloc((void**)&p->h_st64, sizeof(CgState<double>), hipHostMallocDefault));
    RP_HIP_TRY(hipHostMalloc((void**)&p->h_st32, sizeof(CgState<float>), hipHostMallocDefault));
    RP_HIP_TRY(hipHostMalloc((void**)&p->h_st_outer, sizeof(CgState<double>), hipHostMallocDefault));
    RP_TRY(dalloc(&p->d_bi_st, 1));
    RP_HIP_TRY(hipMemset(p->d_bi_st, 0, sizeof(BiState)));
    RP_HIP_TRY(hipHostMalloc((void**)&p->h_bi_st, sizeof(BiState), hipHostMallocDefault));
    RP_HIP_TRY(hipHostMalloc((void**)&p->h_flags, 2 * sizeof(uint32_t), hipHostMallocDefault));
    RP_HIP_TRY(hipMalloc((void**)&p->d_src, sizeof(const double*) * 4 * (size_t)std::max(p->alpha, 1)));
    return RP_OK;
}

// true when ptr is device memory (hipMalloc) reachable from the plan's GPU
bool is_device_ptr(const void* ptr) {
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int activate(rp_plan* p) {
    int cur = -1;
    RP_HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) RP_HIP_TRY(hipSetDevice(p->device));
    return RP_OK;
}

#define RP_CHECK(cond, code, ...)       \
    do {                                \
        if (!(cond)) {                  \
            ::rp::set_error(__VA_ARGS__); \
            return (code);              \
        }                               \
    } while (0)

int create(int32_t n_ranks_total, const int32_t* n_cells_all, int32_t first, int32_t alpha,
           const rp_rank_desc* share, rp_plan** out) {
    RP_CHECK(out != nullptr, RP_ERR_ARG, "out is NULL");
    *out = nullptr;
    RP_CHECK(n_ranks_total >= 1 && n_cells_all != nullptr, RP_ERR_ARG, "need n_ranks_total >= 1 and n_cells_all");
    RP_CHECK(alpha >= 1 && first >= 0 && (int64_t)first + alpha <= n_ranks_total, RP_ERR_ARG,
             "share [%d, %d + %d) is not inside the %d ranks", first, first, alpha, n_ranks_total);
    RP_CHECK(share != nullptr, RP_ERR_ARG, "share is NULL");

    std::unique_ptr<rp_plan, void (*)(rp_plan*)> p(new (std::nothrow) rp_plan(), free_plan);
    RP_CHECK(p != nullptr, RP_ERR_ARG, "out of host memory");
    p->n_ranks_total = n_ranks_total;
    p->first = first;
    p->alpha = alpha;
    p->off_all.assign(n_ranks_total + 1, 0);
    for (int32_t r = 0; r < n_ranks_total; ++r) {
        RP_CHECK(n_cells_all[r] >= 0, RP_ERR_ARG, "n_cells_all[%d] < 0", r);
        p->off_all[r + 1] = p->off_all[r] + n_cells_all[r];
    }
    int64_t slots = 0, rows = 0, ifaces = 0;
    p->slot_off.assign(alpha + 1, 0);
    p->row0.assign(alpha + 1, 0);
    p->iface_off.assign(alpha + 1, 0);
    for (int32_t s = 0; s < alpha; ++s) {
        const rp_rank_desc& d = share[s];
        RP_CHECK(d.n_cells == n_cells_all[first + s], RP_ERR_ARG,
                 "share[%d].n_cells = %d but n_cells_all[%d] = %d", s, d.n_cells, first + s,
                 n_cells_all[first + s]);
        RP_CHECK(d.n_faces >= 0 && d.n_iface >= 0, RP_ERR_ARG, "share[%d]: negative count", s);
        RP_CHECK(d.n_faces == 0 || (d.owner && d.neighbour), RP_ERR_ARG, "share[%d]: owner/neighbour NULL", s);
        RP_CHECK(d.n_iface == 0 || (d.iface_cell && d.iface_nbr_rank && d.iface_nbr_cell), RP_ERR_ARG,
                 "share[%d]: interface arrays NULL", s);
        slots += (int64_t)d.n_cells + 2 * (int64_t)d.n_faces + d.n_iface;
        rows += d.n_cells;
        ifaces += d.n_iface;
        RP_CHECK(slots < INT32_MAX && rows < INT32_MAX && ifaces < INT32_MAX, RP_ERR_OVERFLOW,
                 "the share's rows or slots reach 2^31");
        p->slot_off[s + 1] = (int32_t)slots;
        p->row0[s + 1] = (int32_t)rows;
        p->iface_off[s + 1] = (int32_t)ifaces;
        p->n_cells.push_back(d.n_cells);
        p->n_faces.push_back(d.n_faces);
        p->n_iface.push_back(d.n_iface);
    }
    p->n_rows = rows;
    p->n_slots = slots;
    // everything above is host-side validation; the GPU is touched from here on
    RP_HIP_TRY(hipGetDevice(&p->device));
    RP_TRY(plan_build(p.get(), share));
    RP_TRY(alloc_values(p.get()));
    p->h_src.assign(4 * (size_t)alpha, nullptr);
    *out = p.release();
    return RP_OK;
}

int update(rp_plan* p, const double* const* diag, const double* const* upper, const double* const* lower,
           const double* const* iface, hipStream_t s) {
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(diag && upper && iface, RP_ERR_ARG, "diag/upper/iface pointer arrays are NULL");
    RP_TRY(activate(p));
    bool all_device = true;
    for (int32_t i = 0; i < p->alpha; ++i) {
        RP_CHECK(p->n_cells[i] == 0 || diag[i], RP_ERR_ARG, "diag[%d] is NULL", i);
        RP_CHECK(p->n_faces[i] == 0 || upper[i], RP_ERR_ARG, "upper[%d] is NULL", i);
        RP_CHECK(p->n_faces[i] == 0 || !lower || lower[i], RP_ERR_ARG, "lower[%d] is NULL", i);
        RP_CHECK(p->n_iface[i] == 0 || iface[i], RP_ERR_ARG, "iface[%d] is NULL", i);
        const double* ptrs[4] = {diag[i], upper[i], lower ? lower[i] : nullptr, iface[i]};
        for (const double* q : ptrs)
            if (q && !is_device_ptr(q)) all_device = false;
        p->h_src[4 * i + 0] = diag[i];
        p->h_src[4 * i + 1] = upper[i];
        p->h_src[4 * i + 2] = lower ? lower[i] : upper[i];
        p->h_src[4 * i + 3] = iface[i];
    }
    RP_TRY(launch_clear_flags(p->d_flags, s));
    if (all_device) {
        // the receive buffer stays virtual: the reorder reads every slot from
        // its rank's array through the pointer table
        RP_HIP_TRY(hipMemcpyAsync(p->d_src, p->h_src.data(), sizeof(const double*) * 4 * (size_t)p->alpha,
                                  hipMemcpyHostToDevice, s));
        RP_TRY(launch_update_gather(p, p->d_src, lower != nullptr, p->d_flags, s));
    } else {
        // host-buffer path: one copy per rank array into the receive buffer at U's offsets
        for (int32_t i = 0; i < p->alpha; ++i) {
            double* dst = p->d_recv + p->slot_off[i];
            const size_t nc = p->n_cells[i], nf = p->n_faces[i], ni = p->n_iface[i];
            if (nc) RP_HIP_TRY(hipMemcpyAsync(dst, diag[i], nc * 8, hipMemcpyDefault, s));
            if (nf) RP_HIP_TRY(hipMemcpyAsync(dst + nc, upper[i], nf * 8, hipMemcpyDefault, s));
            if (nf) RP_HIP_TRY(hipMemcpyAsync(dst + nc + nf, lower ? lower[i] : upper[i], nf * 8,
                                              hipMemcpyDefault, s));
            if (ni) RP_HIP_TRY(hipMemcpyAsync(dst + nc + 2 * nf, iface[i], ni * 8, hipMemcpyDefault, s));
        }
        RP_TRY(launch_symmetry_check(p, p->d_recv, lower != nullptr, s));
        RP_TRY(launch_update(p, p->d_recv, s));
    }
    p->has_values = true;
    p->values_version += 1;
    p->last_stream = s;
    return RP_OK;
}

}  // namespace
}  // namespace rp

using namespace rp;

extern "C" {

int rp_plan_create(int32_t n_ranks_total, const int32_t* n_cells_all, int32_t first_rank, int32_t alpha,
                   const rp_rank_desc* share, rp_plan** out) {
    clear_error();
    try {
        return create(n_ranks_total, n_cells_all, first_rank, alpha, share, out);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return RP_ERR_ARG;
    }
}

void rp_plan_destroy(rp_plan* plan) {
    if (!plan) return;
    (void)hipDeviceSynchronize();
    free_plan(plan);
}

int rp_plan_sizes(const rp_plan* p, int64_t* n_rows, int64_t* nnz_local, int64_t* nnz_nonlocal,
                  int64_t* n_slots, int64_t* slot_off) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    if (n_rows) *n_rows = p->n_rows;
    if (nnz_local) *nnz_local = p->nnz;
    if (nnz_nonlocal) *nnz_nonlocal = p->nnz_nl;
    if (n_slots) *n_slots = p->n_slots;
    if (slot_off)
        for (int32_t i = 0; i <= p->alpha; ++i) slot_off[i] = p->slot_off[i];
    return RP_OK;
}

int rp_plan_spmv_windows(const rp_plan* p, int32_t* mode, int32_t* offsets, int32_t* enabled) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    if (mode) *mode = p->xw_found;
    if (offsets) {
        offsets[0] = p->xw_d[0];
        offsets[1] = p->xw_d[1];
    }
    if (enabled) *enabled = p->xw_mode == p->xw_found && p->xw_found >= 0;
    return RP_OK;
}

int rp_plan_set_spmv_windows(rp_plan* p, int32_t enable) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    p->xw_mode = enable ? p->xw_found : -1;
    return RP_OK;
}

int rp_plan_spmv_format(const rp_plan* p, rp_spmv_format* info) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(info != nullptr, RP_ERR_ARG, "info is NULL");
    const bool coded = p->goi_on && p->coded_groups > 0;
    const int64_t n = p->n_rows;
    const int64_t cg = coded ? p->coded_groups : 0, cr = coded ? p->coded_rows : 0, cn = coded ? p->coded_nnz : 0;
    // values, index words (coded: mask per row, k + offset table and the
    // first row pointer per group; CSR: col per entry, row pointer per row),
    // x read once, y written once, the closing row pointer
    auto bytes = [&](int64_t sv) {
        return cn * sv + 2 * cr + 4 * (1 + rp::GOI_KMAX) * cg + 4 * cg + (p->nnz - cn) * (sv + 4) + 4 * (n - cr) +
               2 * n * sv + 4;
    };
    info->enabled = p->goi_on;
    info->reserved = 0;
    info->n_groups = p->n_groups;
    info->coded_groups = p->coded_groups;
    info->coded_rows = p->coded_rows;
    info->coded_nnz = p->coded_nnz;
    info->bytes64 = bytes(8);
    info->bytes32 = bytes(4);
    return RP_OK;
}

int rp_plan_set_spmv_format(rp_plan* p, int32_t enable) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    p->goi_on = enable ? 1 : 0;
    return RP_OK;
}

int rp_plan_get_csr(rp_plan* p, int32_t* row_ptr, int32_t* col, int32_t* perm, int32_t* nl_row_ptr,
                    int64_t* nl_col) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_TRY(activate(p));
    RP_HIP_TRY(hipDeviceSynchronize());
    if (row_ptr) RP_HIP_TRY(hipMemcpy(row_ptr, p->d_row_ptr, 4 * (p->n_rows + 1), hipMemcpyDeviceToHost));
    if (col && p->nnz) RP_HIP_TRY(hipMemcpy(col, p->d_col, 4 * p->nnz, hipMemcpyDeviceToHost));
    if (perm && p->n_slots) RP_HIP_TRY(hipMemcpy(perm, p->d_perm, 4 * p->n_slots, hipMemcpyDeviceToHost));
    if (nl_row_ptr)
        RP_HIP_TRY(hipMemcpy(nl_row_ptr, p->d_nl_row_ptr, 4 * (p->n_rows + 1), hipMemcpyDeviceToHost));
    if (nl_col && p->nnz_nl) RP_HIP_TRY(hipMemcpy(nl_col, p->d_nl_col, 8 * p->nnz_nl, hipMemcpyDeviceToHost));
    return RP_OK;
}

int rp_plan_device_ptrs(const rp_plan* p, rp_device_ptrs* out) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(out != nullptr, RP_ERR_ARG, "out is NULL");
    out->row_ptr = p->d_row_ptr;
    out->col = p->d_col;
    out->perm = p->d_perm;
    out->nl_row_ptr = p->d_nl_row_ptr;
    out->nl_col = p->d_nl_col;
    out->val64 = p->d_val64;
    out->val32 = p->d_val32;
    out->dinv64 = p->d_dinv64;
    out->dinv32 = p->d_dinv32;
    out->recv = p->d_recv;
    return RP_OK;
}

int rp_plan_block_jacobi(rp_plan* p, int32_t block_size, int64_t* n_blocks, int32_t* start, double* minv64,
                         float* minv32) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(p->has_values, RP_ERR_ARG, "no values yet: call rp_update_values first");
    RP_TRY(activate(p));
    hipStream_t s = p->last_stream;
    RP_TRY(bj_prepare(p, block_size, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    const int64_t nb = p->bj_blocks, P = (int64_t)block_size * (block_size + 1) / 2;
    if (n_blocks) *n_blocks = nb;
    if (start) RP_HIP_TRY(hipMemcpy(start, p->d_bj_start, sizeof(int32_t) * (nb + 1), hipMemcpyDeviceToHost));
    if (minv64 && nb) RP_HIP_TRY(hipMemcpy(minv64, p->d_bj_minv64, sizeof(double) * nb * P, hipMemcpyDeviceToHost));
    if (minv32 && nb) RP_HIP_TRY(hipMemcpy(minv32, p->d_bj_minv32, sizeof(float) * nb * P, hipMemcpyDeviceToHost));
    return RP_OK;
}

int rp_plan_amg_setup(rp_plan* p, void* stream) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(p->has_values, RP_ERR_ARG, "no values yet: call rp_update_values first");
    RP_TRY(activate(p));
    hipStream_t s = as_stream(stream);
    RP_TRY(values_solvable(p, s));
    RP_TRY(amg_setup(p, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    return RP_OK;
}

int rp_plan_amg_levels(const rp_plan* p, int32_t* n_levels) {
    clear_error();
    RP_CHECK(p != nullptr && n_levels != nullptr, RP_ERR_ARG, "plan or n_levels is NULL");
    *n_levels = p->amg ? p->amg->n_levels : 0;
    return RP_OK;
}

int rp_plan_amg_level(const rp_plan* pc, int32_t level, int64_t* n, int64_t* nnz, int32_t* row_ptr, int32_t* col,
                      double* val, double* dinv, int32_t* agg, int32_t* mem_ptr, int32_t* mem) {
    clear_error();
    RP_CHECK(pc != nullptr, RP_ERR_ARG, "plan is NULL");
    rp_plan* p = const_cast<rp_plan*>(pc);
    RP_CHECK(p->amg != nullptr && level >= 0 && level < p->amg->n_levels, RP_ERR_ARG,
             "level %d outside the hierarchy (%d levels)", level, p->amg ? p->amg->n_levels : 0);
    RP_TRY(activate(p));
    RP_HIP_TRY(hipDeviceSynchronize());
    const AmgHier& h = *p->amg;
    const AmgLevel& L = h.lev[level];
    const int64_t ln = L.n, lnnz = L.nnz;
    if (n) *n = ln;
    if (nnz) *nnz = lnnz;
    const int32_t* drp = level == 0 ? p->d_row_ptr : L.row_ptr;
    const int32_t* dcol = level == 0 ? p->d_col : L.col;
    const double* dval = level == 0 ? p->d_val64 : L.val64;
    const double* ddinv = level == 0 ? p->d_dinv64 : L.dinv64;
    if (row_ptr) RP_HIP_TRY(hipMemcpy(row_ptr, drp, sizeof(int32_t) * (ln + 1), hipMemcpyDeviceToHost));
    if (col && lnnz) RP_HIP_TRY(hipMemcpy(col, dcol, sizeof(int32_t) * lnnz, hipMemcpyDeviceToHost));
    if (val && lnnz) RP_HIP_TRY(hipMemcpy(val, dval, sizeof(double) * lnnz, hipMemcpyDeviceToHost));
    if (dinv && ln) RP_HIP_TRY(hipMemcpy(dinv, ddinv, sizeof(double) * ln, hipMemcpyDeviceToHost));
    if (level + 1 < h.n_levels) {
        const int64_t nc = h.lev[level + 1].n;
        if (agg && ln) RP_HIP_TRY(hipMemcpy(agg, L.agg, sizeof(int32_t) * ln, hipMemcpyDeviceToHost));
        if (mem_ptr) RP_HIP_TRY(hipMemcpy(mem_ptr, L.mem_ptr, sizeof(int32_t) * (nc + 1), hipMemcpyDeviceToHost));
        if (mem && ln) RP_HIP_TRY(hipMemcpy(mem, L.mem, sizeof(int32_t) * ln, hipMemcpyDeviceToHost));
    }
    return RP_OK;
}

int rp_plan_amg_coarse_inverse(const rp_plan* pc, double* cinv) {
    clear_error();
    RP_CHECK(pc != nullptr && cinv != nullptr, RP_ERR_ARG, "plan or cinv is NULL");
    rp_plan* p = const_cast<rp_plan*>(pc);
    RP_CHECK(p->amg != nullptr, RP_ERR_ARG, "no multigrid hierarchy yet");
    RP_TRY(activate(p));
    RP_HIP_TRY(hipDeviceSynchronize());
    const int64_t nL = p->amg->lev[p->amg->n_levels - 1].n;
    RP_HIP_TRY(hipMemcpy(cinv, p->amg->cinv64, sizeof(double) * nL * nL, hipMemcpyDeviceToHost));
    return RP_OK;
}

int rp_plan_amg_apply(rp_plan* p, const double* r, double* z, void* stream) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(p->has_values, RP_ERR_ARG, "no values yet: call rp_update_values first");
    RP_CHECK(p->n_rows == 0 || (r != nullptr && z != nullptr), RP_ERR_ARG, "r or z is NULL");
    RP_TRY(activate(p));
    hipStream_t s = as_stream(stream);
    RP_TRY(values_solvable(p, s));
    RP_TRY(amg_prepare(p, false, s));
    if (p->n_rows == 0) return RP_OK;
    return amg_apply<double>(p, r, z, nullptr, 0, false, nullptr, s);
}

int rp_plan_set_vec_grid(rp_plan* p, int32_t blocks) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(blocks >= 0 && blocks <= VEC_GRID_LIMIT, RP_ERR_ARG, "blocks must be in 0..%d", VEC_GRID_LIMIT);
    p->vec_grid_override = blocks;
    return RP_OK;
}

int rp_plan_get_values(rp_plan* p, double* val64, float* val32, double* dinv64, float* dinv32) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(p->has_values, RP_ERR_ARG, "no values yet: call rp_update_values first");
    RP_TRY(activate(p));
    RP_HIP_TRY(hipDeviceSynchronize());
    if (val64 && p->n_slots) RP_HIP_TRY(hipMemcpy(val64, p->d_val64, 8 * p->n_slots, hipMemcpyDeviceToHost));
    if (val32 && p->n_slots) RP_HIP_TRY(hipMemcpy(val32, p->d_val32, 4 * p->n_slots, hipMemcpyDeviceToHost));
    if (dinv64 && p->n_rows) RP_HIP_TRY(hipMemcpy(dinv64, p->d_dinv64, 8 * p->n_rows, hipMemcpyDeviceToHost));
    if (dinv32 && p->n_rows) RP_HIP_TRY(hipMemcpy(dinv32, p->d_dinv32, 4 * p->n_rows, hipMemcpyDeviceToHost));
    return RP_OK;
}

int rp_update_values(rp_plan* p, const double* const* diag, const double* const* upper,
                     const double* const* lower, const double* const* iface, void* stream) {
    clear_error();
    return update(p, diag, upper, lower, iface, as_stream(stream));
}

int rp_update_values_slots(rp_plan* p, const double* slots, void* stream) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(slots != nullptr || p->n_slots == 0, RP_ERR_ARG, "slots is NULL");
    RP_TRY(activate(p));
    hipStream_t s = as_stream(stream);
    RP_TRY(launch_clear_flags(p->d_flags, s));
    RP_TRY(launch_symmetry_check(p, slots, true, s));
    RP_TRY(launch_update(p, slots, s));
    p->has_values = true;
    p->values_version += 1;
    p->last_stream = s;
    return RP_OK;
}

int rp_spmv(rp_plan* p, int32_t precision, const void* x, void* y, void* stream) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(p->has_values, RP_ERR_ARG, "no values yet: call rp_update_values first");
    RP_CHECK(p->n_rows == 0 || (x && y), RP_ERR_ARG, "x or y is NULL");
    RP_CHECK(precision == RP_FP64 || precision == RP_FP32, RP_ERR_ARG, "precision must be RP_FP64 or RP_FP32");
    RP_TRY(activate(p));
    if (precision == RP_FP64)
        return launch_spmv64(p, static_cast<const double*>(x), static_cast<double*>(y), as_stream(stream));
    return launch_spmv32(p, static_cast<const float*>(x), static_cast<float*>(y), as_stream(stream));
}

void rp_solve_opts_default(rp_solve_opts* o) {
    if (!o) return;
    o->tol = 1e-8;
    o->inner_tol = 1e-4;
    o->update_delta = 0.1;
    o->max_iter = 100000;
    o->precision = RP_FP64;
    o->max_outer = 200;
    o->check_every = 32;
    o->x0_zero = 0;
    o->max_restarts = 5;
    o->method = RP_CG;
    o->transpose = 0;
    o->graph = 0;
    o->precond = RP_PRECOND_JACOBI;
    o->block_size = 4;
    o->fused_loop = RP_LOOP_AUTO;
}

int rp_solve(rp_plan* p, const double* b, double* x, const rp_solve_opts* opts, rp_solve_info* info,
             void* stream) {
    clear_error();
    rp_solve_info local_info;
    std::memset(&local_info, 0, sizeof(local_info));
    rp_solve_info& inf = info ? *info : local_info;
    std::memset(&inf, 0, sizeof(inf));
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    rp_solve_opts o;
    rp_solve_opts_default(&o);
    if (opts) o = *opts;
    RP_CHECK(p->n_rows == 0 || (b && x), RP_ERR_ARG, "b or x is NULL");
    RP_CHECK(o.tol >= 0.0 && o.inner_tol > 0.0 && o.inner_tol < 1.0 && o.update_delta > 0.0 &&
                 o.update_delta < 1.0 && o.max_iter >= 0 && o.max_outer >= 0 && o.max_restarts >= 0,
             RP_ERR_ARG, "bad solve options");
    RP_CHECK(o.precision == RP_FP64 || o.precision == RP_MIXED || o.precision == RP_MIXED_RR, RP_ERR_ARG,
             "precision must be RP_FP64, RP_MIXED or RP_MIXED_RR");
    RP_CHECK(o.method == RP_CG || o.method == RP_BICGSTAB, RP_ERR_ARG, "method must be RP_CG or RP_BICGSTAB");
    RP_CHECK(o.method == RP_CG || o.precision == RP_FP64, RP_ERR_UNSUPPORTED, "BiCGStab runs in FP64 only");
    RP_CHECK(o.transpose == 0 || o.transpose == 1, RP_ERR_ARG, "transpose must be 0 or 1");
    RP_CHECK(o.graph == 0 || o.graph == 1, RP_ERR_ARG, "graph must be 0 or 1");
    RP_CHECK(o.fused_loop == RP_LOOP_AUTO || o.fused_loop == RP_LOOP_COOPERATIVE || o.fused_loop == RP_LOOP_THREE,
             RP_ERR_ARG, "fused_loop must be RP_LOOP_AUTO, RP_LOOP_COOPERATIVE or RP_LOOP_THREE");
    RP_CHECK(o.precond == RP_PRECOND_JACOBI || o.precond == RP_PRECOND_BLOCK_JACOBI || o.precond == RP_PRECOND_AMG,
             RP_ERR_ARG, "precond must be RP_PRECOND_JACOBI, RP_PRECOND_BLOCK_JACOBI or RP_PRECOND_AMG");
    RP_CHECK(o.precond == RP_PRECOND_JACOBI || (o.block_size >= 1 && o.block_size <= RP_BJ_MAX_BLOCK), RP_ERR_ARG,
             "block_size must be in 1..%d", RP_BJ_MAX_BLOCK);
    RP_CHECK(o.precond == RP_PRECOND_JACOBI || o.method == RP_CG, RP_ERR_UNSUPPORTED,
             "block-Jacobi is built for CG (RP_CG) only");
    RP_CHECK(o.precond != RP_PRECOND_BLOCK_JACOBI || p->ro_mode == 0, RP_ERR_UNSUPPORTED,
             "block-Jacobi runs in the fused row order only (solve order 0)");
    RP_TRY(activate(p));
    hipStream_t s = as_stream(stream);
    p->last_stream = s;
    int rc;
    if (p->n_rows == 0) {
        rc = RP_OK;
    } else if (p->ro_mode == 1) {
        rc = solve_in_order(p, b, x, o, inf, s);
    } else if (o.method == RP_BICGSTAB) {
        rc = solve_bicgstab(p, b, x, o, inf, s);
    } else if (o.precision == RP_FP64) {
        rc = solve_fp64(p, b, x, o, inf, s);
    } else {
        rc = solve_mixed(p, b, x, o, inf, s, o.precision == RP_MIXED_RR);
    }
    inf.status = rc;
    return rc;
}

int rp_plan_set_solve_order(rp_plan* p, int32_t mode) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(mode == 0 || mode == 1, RP_ERR_ARG, "solve order must be 0 (fused) or 1 (reverse Cuthill-McKee)");
    RP_CHECK(mode == 0 || p->nnz_nl == 0, RP_ERR_UNSUPPORTED,
             "the solve order needs a share without non-local entries");
    RP_TRY(activate(p));
    if (mode == 1 && p->d_ro_perm == nullptr && p->n_rows > 0) {
        RP_HIP_TRY(hipDeviceSynchronize());
        RP_TRY(order_build(p));
    }
    p->ro_mode = mode;
    return RP_OK;
}

int rp_plan_solve_order(const rp_plan* p, int32_t* mode, int32_t* perm) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    if (mode) *mode = p->ro_mode;
    if (perm) {
        RP_CHECK(p->ro_mode == 1 || !p->h_ro_perm.empty(), RP_ERR_ARG,
                 "no solve order built (rp_plan_set_solve_order(plan, 1) first)");
        std::copy(p->h_ro_perm.begin(), p->h_ro_perm.end(), perm);
    }
    return RP_OK;
}

int rp_rcm_order(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* perm) {
    clear_error();
    RP_CHECK(n >= 0 && (n == 0 || (row_ptr && perm)), RP_ERR_ARG, "bad arguments");
    RP_CHECK(row_ptr == nullptr || row_ptr[0] == 0, RP_ERR_ARG, "row_ptr[0] must be 0");
    for (int32_t i = 0; i < n; ++i) RP_CHECK(row_ptr[i + 1] >= row_ptr[i], RP_ERR_ARG, "row_ptr decreases");
    const int64_t nnz = n > 0 ? row_ptr[n] : 0;
    RP_CHECK(nnz == 0 || col != nullptr, RP_ERR_ARG, "col is NULL");
    for (int64_t j = 0; j < nnz; ++j) RP_CHECK(col[j] >= 0 && col[j] < n, RP_ERR_ARG, "column out of range");
    const std::vector<int32_t> o = rcm_order(n, row_ptr, col);
    std::copy(o.begin(), o.end(), perm);
    return RP_OK;
}

int rp_value_grad(rp_plan* p, const double* lambda, const double* x, double* g_slots, void* stream) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(p->n_rows == 0 || (lambda && x && g_slots), RP_ERR_ARG, "lambda, x or g_slots is NULL");
    RP_CHECK(p->nnz_nl == 0, RP_ERR_UNSUPPORTED, "value gradients need a share without non-local entries");
    RP_TRY(activate(p));
    return launch_value_grad(p, lambda, x, g_slots, as_stream(stream));
}

int rp_sync(rp_plan* p) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_TRY(activate(p));
    hipStream_t s = p->last_stream;
    RP_HIP_TRY(hipStreamSynchronize(s));
    RP_TRY(timing_collect(p, RP_KERNEL_SCATTER, INT64_MAX));
    RP_HIP_TRY(hipMemcpy(p->h_flags, p->d_flags, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (p->h_flags[0] & FLAG_VALUE) {
        set_error("the last update produced a value that is not finite or a diagonal <= 0");
        return RP_ERR_VALUE;
    }
    return RP_OK;
}

const char* rp_last_error(void) { return g_err; }

int rp_plan_set_timing(rp_plan* p, int32_t enable) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_TRY(activate(p));
    RP_HIP_TRY(hipDeviceSynchronize());
    RP_CHECK(enable >= 0, RP_ERR_ARG, "enable must be 0 (off) or the stride of the recorded launches (>= 1)");
    p->timing.enabled = enable != 0;
    p->timing.stride = enable > 0 ? enable : 1;
    for (int k = 0; k < RP_N_KERNELS; ++k) {
        p->timing.launches[k] = 0;
        p->timing.total_ms[k] = 0.0;
        EventPool& e = p->timing.pool[k];
        e.used = 0;
        e.seen = 0;
        e.chunk0 = 0;
        e.open = false;
    }
    return RP_OK;
}

int rp_plan_kernel_stats(rp_plan* p, int32_t kernel, int64_t* launches, double* total_ms) {
    clear_error();
    RP_CHECK(p != nullptr, RP_ERR_ARG, "plan is NULL");
    RP_CHECK(kernel >= 0 && kernel < RP_N_KERNELS, RP_ERR_ARG, "unknown kernel id %d", kernel);
    RP_TRY(activate(p));
    RP_HIP_TRY(hipDeviceSynchronize());
    RP_TRY(timing_collect(p, kernel, INT64_MAX));
    if (launches) *launches = p->timing.launches[kernel];
    if (total_ms) *total_ms = p->timing.total_ms[kernel];
    return RP_OK;
}

}  // extern "C"

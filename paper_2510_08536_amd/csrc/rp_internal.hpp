// Internal declarations of librp: the plan object, error plumbing and the
// launchers each kernel file provides.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rp.h"

namespace rp {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

#define RP_HIP_TRY(call)                                                          \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::rp::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                  \
            return RP_ERR_HIP;                                                    \
        }                                                                         \
    } while (0)

#define RP_TRY(expr)              \
    do {                          \
        int rc_ = (expr);         \
        if (rc_ != RP_OK) return rc_; \
    } while (0)

// device-side error bits (plan->d_flags[0])
enum : uint32_t {
    FLAG_MESH_RANGE = 1u << 0,     // owner/neighbour/interface index out of range
    FLAG_MESH_SELF = 1u << 1,      // owner == neighbour, or interface to own rank
    FLAG_MESH_DUP = 1u << 2,       // a matrix entry addressed twice
    FLAG_MESH_UNPAIRED = 1u << 3,  // interface coupling without its partner
    FLAG_VALUE = 1u << 8,          // non-finite value or diag <= 0 in an update
};
// plan->d_flags[1]: set when the last update produced a non-symmetric matrix
// (upper != lower, or an interface value != its partner's)

// ---------------------------------------------------------------------------
// CG state kept on the device; S is the scalar type of the iteration.
//
// Reductions need no atomics or fences: a kernel leaves one partial sum per
// block, and every block of the next kernel adds all of them in index order
// (so all blocks hold the same scalar).  Scalars that a later kernel of the
// same iteration still reads while block 0 stores the next value live in a
// ring indexed by the iteration number, which the host passes to each kernel.
// ---------------------------------------------------------------------------
enum : int32_t {
    CG_RUNNING = 0,
    CG_CONVERGED = 1,   // recurrence residual passed the threshold
    CG_BREAKDOWN = 2,   // p.Ap <= 0, (r, z) <= 0 or not finite
    CG_ZERO_RHS = 4,    // ||b|| = 0
    CG_PAUSED = 5,      // residual fell below pause_thresh: FP64 update due
    BI_HALF = 6,        // BiCGStab: ||s|| small at the half step of iteration half_k;
                        // that iteration's last kernel adds alpha y, then the solve ends
};

template <typename S>
struct CgState {
    S rz[4];        // rz[k & 3] = (r_k, M^-1 r_k)
    S alpha, beta, pq;
    S rr;           // (r, r) of the latest residual
    S bb;           // (b, b)
    S thresh;       // tol^2 * bb: convergence of the recurrence residual
    S rr_true;      // (r, r) of the last explicit residual b - A x
    S rr_ref;       // (r, r) when the FP32 iteration last took an FP64 update
    S pause_frac2;  // update_delta^2 (0: never pause)
    S pause_thresh; // pause_frac2 * rr_ref
    int32_t iter;   // completed iterations
    int32_t done;   // CG_*
    int32_t max_iter;  // iteration budget (kernels past it do nothing)
    int32_t kk;        // iteration K2 works on, for K3 (-1: budget spent)
};

// Device-side scalars of one BiCGStab solve (FP64)
struct BiState {
    double rho[4];  // rho[k & 3] = (rh, r_k), written by iteration k
    double alpha, omega;
    double rr;      // (r, r) of the latest residual
    double bb;      // (b, b)
    double thresh;  // tol^2 * bb
    double rr_true; // (r, r) of the last explicit residual b - A x
    int32_t iter;   // completed iterations
    int32_t done;   // CG_* / BI_HALF
    int32_t half_k; // iteration whose half step stopped (valid while done == BI_HALF)
    int32_t pad;
};

// partial-sum regions of plan->d_partials (counted in elements of S)
// kernel launch shapes
constexpr int SPMV_BLOCK = 256;               // rows per SpMV block = threads
constexpr int SPMV_UNROLL = 8;                // staged products per thread
constexpr int SPMV_CAP = SPMV_UNROLL * SPMV_BLOCK;
constexpr int SPMV_PAD = 4;                   // zeroed col / val elements past the end (pack loads)
constexpr int GOI_KMAX = 16;                  // offsets per offset-coded SpMV group (mask width)
constexpr int VEC_BLOCK = 256;                // elementwise kernels
// grid-stride elements a thread of K2 (r update) / K3 (x, p update) loads
// per trip, measured best per kernel on MI355X: 4 / 4 for FP64, 2 / 1 for FP32
template <typename T>
constexpr int vec_unroll_r() { return sizeof(T) == 8 ? 4 : 2; }
template <typename T>
constexpr int vec_unroll_xp() { return sizeof(T) == 8 ? 4 : 1; }
constexpr int N_XCD = 8;                      // MI355X: 8 accelerator dies
constexpr int BJ_MAX = RP_BJ_MAX_BLOCK;       // largest block-Jacobi block

// ---------------------------------------------------------------------------
// aggregation multigrid hierarchy (amg.hip)
// ---------------------------------------------------------------------------
constexpr int AMG_MAX_LEVELS = 40;
constexpr int AMG_COARSE_MAX = RP_AMG_COARSE_MAX;   // rows of the coarsest level (dense inverse)
constexpr int AMG_ROUNDS = 16;        // matching rounds per level at most

struct AmgLevel {
    int64_t n = 0, nnz = 0;
    // levels >= 1 (level 0 is the plan's fused CSR and values)
    int32_t* row_ptr = nullptr;   // [n + 1]
    int32_t* col = nullptr;       // [nnz + SPMV_PAD]
    double* val64 = nullptr;      // [nnz + SPMV_PAD]
    float* val32 = nullptr;       // RNE copy
    double* dinv64 = nullptr;     // [n] 1 / diagonal
    float* dinv32 = nullptr;
    int32_t* diag_pos = nullptr;  // [n] position of the diagonal entry
    // all levels but the coarsest: the aggregates and the next level's map
    int32_t* agg = nullptr;       // [n] coarse row of each row
    int32_t* mem_ptr = nullptr;   // [n_c + 1] members of each coarse row,
    int32_t* mem = nullptr;       // [n]       ascending
    int32_t* cptr = nullptr;      // [nnz_c + 1] coarse entry e sums the values at
    int32_t* cpos = nullptr;      // [nnz]       positions cpos[cptr[e] .. cptr[e+1])
    // V-cycle vectors per precision: in (levels >= 1), x and t (smoothed
    // levels), out (levels >= 1)
    double* vec64[4] = {nullptr, nullptr, nullptr, nullptr};
    float* vec32[4] = {nullptr, nullptr, nullptr, nullptr};
};

struct AmgHier {
    int32_t n_levels = 0;
    AmgLevel lev[AMG_MAX_LEVELS];
    double* cinv64 = nullptr;     // [n_L^2] inverse of the coarsest matrix, row-major
    float* cinv32 = nullptr;      // RNE copy
    double* cwork = nullptr;      // [n_L^2] elimination work
    uint32_t* flag = nullptr;     // [2] pair counter / error bits
    int64_t version = -1;         // values_version the coarse values belong to
    // the V-cycle below tail_level runs in one workgroup (amg.hip); its
    // per-level pointers per precision, on the device
    int32_t tail_level = 0;       // 0: none
    void* tail64 = nullptr;
    void* tail32 = nullptr;
};

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct EventPool {
    std::vector<hipEvent_t> start, stop;
    std::vector<int64_t> idx;   // launch of each recorded pair, counted from the chunk's first
    int64_t used = 0;
    int64_t seen = 0;           // launches since timing was enabled
    int64_t chunk0 = 0;         // `seen` at the last collection
    bool open = false;          // the current launch is being recorded
};

struct Timing {
    bool enabled = false;
    int32_t stride = 1;         // every stride-th launch of a kernel is recorded
    int64_t launches[RP_N_KERNELS] = {0, 0, 0};
    double total_ms[RP_N_KERNELS] = {0, 0, 0};
    EventPool pool[RP_N_KERNELS];
};

}  // namespace rp

struct rp_plan {
    int device = 0;
    int32_t n_ranks_total = 0, first = 0, alpha = 0;
    int64_t n_rows = 0, n_slots = 0, nnz = 0, nnz_nl = 0, n_iface_share = 0;
    std::vector<int64_t> off_all;    // [n_ranks_total+1] global row offsets
    std::vector<int32_t> slot_off;   // [alpha+1] receive-buffer offsets (U)
    std::vector<int32_t> row0;       // [alpha+1] first fused row of each share rank
    std::vector<int32_t> n_cells, n_faces, n_iface;  // per share rank
    std::vector<int32_t> iface_off;  // [alpha+1] offsets into the share's interfaces

    // rank tables on the device
    int32_t* d_slot_off = nullptr;   // [alpha+1]
    int32_t* d_row0 = nullptr;       // [alpha+1]
    int32_t* d_nf = nullptr;         // [alpha] internal faces
    int32_t* d_face_off = nullptr;   // [alpha+1] offsets into the share's faces
    int32_t* d_owner = nullptr;      // [faces] owner cell of each face, rank-local, concatenated
    int32_t* d_nbr = nullptr;        // [faces] neighbour cell of each face
    int32_t* d_iface_off = nullptr;  // [alpha+1]

    // pattern
    int32_t* d_row_ptr = nullptr;    // [n_rows+1]
    int32_t* d_col = nullptr;        // [nnz]
    int32_t* d_perm = nullptr;       // [n_slots] slot -> position (P)
    int32_t* d_perm_inv = nullptr;   // [nnz + nnz_nl] position -> slot
    int32_t* d_nl_row_ptr = nullptr; // [n_rows+1]
    int64_t* d_nl_col = nullptr;     // [nnz_nl]
    int32_t* d_iface_partner = nullptr;  // [n_iface_share] partner slot, -1 if non-local

    // values
    double* d_recv = nullptr;        // [n_slots] receive buffer, slot order
    double* d_val64 = nullptr;       // [n_slots] CSR order (local, then non-local)
    float* d_val32 = nullptr;        // [n_slots]
    double* d_dinv64 = nullptr;      // [n_rows]
    float* d_dinv32 = nullptr;       // [n_rows]
    bool has_values = false;
    int64_t values_version = 0;      // bumped by every update
    double* d_valT = nullptr;        // [nnz + SPMV_PAD] values of A^T (first transposed solve)
    int64_t valT_version = -1;       // values_version d_valT was built from
    uint32_t* d_tflag = nullptr;     // set when an entry has no transposed partner

    // pointer table for device-resident per-rank values: 4*alpha pointers
    // (diag, upper, lower or upper, interface of each share rank)
    const double** d_src = nullptr;
    std::vector<const double*> h_src;

    // solver workspace
    double *d_r = nullptr, *d_p = nullptr, *d_q = nullptr;
    float *d_r32 = nullptr, *d_p32 = nullptr, *d_q32 = nullptr, *d_x32 = nullptr;
    void* d_partials = nullptr;      // [PART_TOTAL] doubles
    rp::CgState<double>* d_st64 = nullptr;
    rp::CgState<float>* d_st32 = nullptr;
    rp::CgState<double>* d_st_outer = nullptr;
    rp::CgState<double>* h_st64 = nullptr;   // pinned mirrors
    rp::CgState<float>* h_st32 = nullptr;
    rp::CgState<double>* h_st_outer = nullptr;
    rp::BiState* d_bi_st = nullptr;          // BiCGStab state and its pinned mirror
    rp::BiState* h_bi_st = nullptr;
    double* d_bi_work = nullptr;             // [5 n_rows] BiCGStab vectors rh, y, s, z, t (first use)
    uint32_t* d_flags = nullptr;     // [2] error bits, asymmetry flag
    uint32_t* h_flags = nullptr;     // pinned mirror

    // offset-coded SpMV index (see spmv.hpp), built with the pattern
    int32_t* d_goi_k = nullptr;      // [groups] offsets per group, 0 = CSR group
    int32_t* d_goi_off = nullptr;    // [groups * GOI_KMAX]
    uint16_t* d_goi_mask = nullptr;  // [n_rows]
    int32_t goi_on = 1;              // the kernels use the coded groups
    int64_t n_groups = 0, coded_groups = 0, coded_rows = 0, coded_nnz = 0;

    // x windows of the SpMV (see spmv.hpp): -1 none, 0 diagonal, 1..2 +-d pairs;
    // xw_mode is what the kernels use: xw_found when enabled, else -1
    int32_t xw_found = -1;
    int32_t xw_mode = -1;
    int32_t xw_d[2] = {0, 0};

    hipStream_t last_stream = nullptr;
    int32_t vec_grid_override = 0;     // rp_plan_set_vec_grid: solver vector-kernel blocks (0 = sized to n)

    // solve order (order.hip): 0 fused rows, 1 reverse Cuthill-McKee
    // renumbering for CG and the mixed solvers (built on first use)
    int32_t ro_mode = 0;
    int32_t* d_ro_perm = nullptr;      // [n_rows] fused row of each solve-order row
    int32_t* d_ro_row_ptr = nullptr;   // [n_rows+1]
    int32_t* d_ro_col = nullptr;       // [nnz + SPMV_PAD] solve-order columns, ascending per row
    int32_t* d_ro_sig = nullptr;       // [nnz] fused CSR position of each solve-order position
    double* d_ro_val64 = nullptr;      // [nnz + SPMV_PAD]
    float* d_ro_val32 = nullptr;       // [nnz + SPMV_PAD]
    double* d_ro_dinv64 = nullptr;     // [n_rows]
    float* d_ro_dinv32 = nullptr;      // [n_rows]
    double *d_ro_b = nullptr, *d_ro_x = nullptr;  // [n_rows] b and x in solve order
    double* d_ro_valT = nullptr;       // [nnz + SPMV_PAD] A^T's values in solve order (first transposed solve)
    int64_t ro_valT_version = -1;      // values_version d_ro_valT was gathered from
    std::vector<int32_t> h_ro_perm;
    int64_t ro_version = -1;           // values_version the solve-order values were gathered from

    // block-Jacobi preconditioner (precond.hip), built on first use for a
    // block size and rebuilt after every update
    int32_t bj_bs = 0;                 // block size of the tables below (0: none)
    bool bj_aligned = false;           // every block starts at a multiple of bs, and bs divides 64
    int64_t bj_blocks = 0;
    int64_t bj_version = -1;           // values_version the inverses were built from
    int32_t* d_bj_start = nullptr;     // [bj_blocks + 1] first fused row of each block
    double* d_bj_minv64 = nullptr;     // [bj_blocks * bs (bs + 1) / 2] packed upper triangles
    float* d_bj_minv32 = nullptr;      // RNE copy
    double* d_z = nullptr;             // [n_rows] z = M^-1 r of the FP64 iteration
    float* d_z32 = nullptr;            // [n_rows] of the FP32 iteration
    uint32_t* d_bj_flag = nullptr;     // set when a block is not positive definite

    uint32_t* d_loop_bar = nullptr;    // abort word and per-block barrier flags of the CG loop (cg_loop.hip)

    rp::AmgHier* amg = nullptr;        // multigrid hierarchy (RP_PRECOND_AMG), built on first use
    rp::AmgHier* amg_ro = nullptr;     // the same on the solve-order copy

    // captured CG iteration chunks (rp_solve_opts.graph), [0] FP64, [1] FP32
    hipStream_t capture_stream = nullptr;
    struct CgGraph {
        hipGraphExec_t exec = nullptr;
        uint64_t key[24] = {};
    } cg_graph[2];
    rp::Timing timing;
};

namespace rp {

// launch-shape helpers
// SpMV-shaped kernels: at most SPMV_GRID_MAX blocks (a multiple of N_XCD),
// block L taking row groups L, L + G, L + 2G, ...
constexpr int SPMV_GRID_MAX = 1536;
inline int spmv_grid(int64_t n_rows) {
    int64_t groups = (n_rows + SPMV_BLOCK - 1) / SPMV_BLOCK;
    // more groups than the cap: the fewest groups per block the cap allows,
    // on just enough blocks that every block gets that many (no short last
    // round on a fraction of the grid)
    const int64_t rounds = (groups + SPMV_GRID_MAX - 1) / SPMV_GRID_MAX;
    if (rounds > 1) groups = (groups + rounds - 1) / rounds;
    int64_t g = ((groups + N_XCD - 1) / N_XCD) * N_XCD;
    if (g < N_XCD) g = N_XCD;
    if (g > SPMV_GRID_MAX) g = SPMV_GRID_MAX;
    return (int)g;
}
// elementwise kernels: grid-stride loops over at most VEC_GRID_MAX blocks
constexpr int VEC_GRID_MAX = 1024;  // 512 and 2048 measured slower for K2/K3
inline int vec_grid(int64_t n) {
    int64_t g = (n + VEC_BLOCK * 4 - 1) / (VEC_BLOCK * 4);
    if (g < 1) g = 1;
    if (g > VEC_GRID_MAX) g = VEC_GRID_MAX;
    return (int)g;
}
// rp_plan_set_vec_grid may raise the solvers' vector grid up to this many
// blocks (far more than the chip holds at once), so that blocks of one launch
// start after others have finished
constexpr int VEC_GRID_LIMIT = 16384;
// the vector grid of the plan's solver kernels
inline int plan_vec_grid(const rp_plan* p) {
    return p->vec_grid_override > 0 ? p->vec_grid_override : vec_grid(p->n_rows);
}
// partial-sum regions (in elements): two SpMV-grid ones, two vector-grid ones
constexpr int PART_A = 0;                                    // pq, or rr of b - A x
constexpr int PART_B = SPMV_GRID_MAX;                        // bb
constexpr int PART_RZ = 2 * SPMV_GRID_MAX;                   // (r, z)
constexpr int PART_RR = 2 * SPMV_GRID_MAX + VEC_GRID_LIMIT;  // (r, r)
constexpr int PART_TOTAL = 2 * SPMV_GRID_MAX + 2 * VEC_GRID_LIMIT;

// plan.hip
int plan_build(rp_plan* p, const rp_rank_desc* share);
// update.hip
// src: the receive buffer in slot order (the plan's own, or the caller's)
int launch_update(rp_plan* p, const double* src, hipStream_t s);
int launch_symmetry_check(rp_plan* p, const double* src, bool lower_given, hipStream_t s);
// device-resident per-rank arrays: symmetry check and reorder by P straight
// from table[4 * alpha] (diag, upper, lower or upper, interface per rank, a
// device array); error bits go to flags[2]
int launch_update_gather(rp_plan* p, const double* const* table, bool lower_given, uint32_t* flags,
                         hipStream_t s);
int launch_clear_flags(uint32_t* flags, hipStream_t s);
// spmv.hip
int launch_spmv64(rp_plan* p, const double* x, double* y, hipStream_t s);
int launch_spmv32(rp_plan* p, const float* x, float* y, hipStream_t s);
// cg.hip
// ordered: run on the solve-order copy (b, x in solve order)
int solve_fp64(rp_plan* p, const double* b, double* x, const rp_solve_opts& o, rp_solve_info& info,
               hipStream_t s, bool ordered = false);
// reliable = true: FP32 PCG with FP64 residual replacement (RP_MIXED_RR);
// false: restarted FP32 inner PCG under FP64 refinement (RP_MIXED)
int solve_bicgstab(rp_plan* p, const double* b, double* x, const rp_solve_opts& o, rp_solve_info& info,
                   hipStream_t s, bool ordered = false);
int build_transpose(rp_plan* p, hipStream_t s);
// values present, no pending value error, symmetric, no non-local block
int values_solvable(rp_plan* p, hipStream_t s);
int solve_mixed(rp_plan* p, const double* b, double* x, const rp_solve_opts& o, rp_solve_info& info,
                hipStream_t s, bool reliable, bool ordered = false);
// precond.hip
// block-Jacobi tables and inverses for block size bs, current for the values
int bj_prepare(rp_plan* p, int32_t bs, hipStream_t s);
// the preconditioned-residual vectors d_z / d_z32
int alloc_z(rp_plan* p);
// amg.hip
// hierarchy from the current values (aggregates, patterns, coarse values);
// ordered: on the solve-order copy instead of the fused pattern
int amg_setup(rp_plan* p, hipStream_t s, bool ordered = false);
// hierarchy present and its values current; V-cycle vectors of one precision
int amg_prepare(rp_plan* p, bool fp32, hipStream_t s, bool ordered = false);
void amg_free(rp_plan* p);
// y = V-cycle(r) on the level-0 system.  part != null: partials of (r, y) ->
// PART_RZ (and, rr, of (r, r) -> PART_RR), n_part of them.  gate != null:
// every kernel returns when *gate < 0.
template <typename T>
int amg_apply(rp_plan* p, const T* r, T* y, T* part, int32_t n_part, bool rr, const int32_t* gate, hipStream_t s,
              bool ordered = false);
// order.hip
// reverse Cuthill-McKee order of a structurally symmetric pattern: perm[k] = row at position k
std::vector<int32_t> rcm_order(int32_t n, const int32_t* row_ptr, const int32_t* col);
int order_build(rp_plan* p);
// CG / mixed / BiCGStab solve on the solve-order copy; b and x in fused order
int solve_in_order(rp_plan* p, const double* b, double* x, const rp_solve_opts& o, rp_solve_info& info,
                   hipStream_t s);
// grad.hip
int launch_value_grad(rp_plan* p, const double* lambda, const double* x, double* g, hipStream_t s);

// timing (capi.cpp)
int timing_begin(rp_plan* p, int kernel, hipStream_t s);
int timing_end(rp_plan* p, int kernel, hipStream_t s);
// fold the first `keep` pending event pairs of `kernel` into the totals and
// drop the rest (launches that found the solve already finished)
int timing_collect(rp_plan* p, int kernel, int64_t keep);

}  // namespace rp

/*
 * rp.h - C ABI of librp.so: matrix repartitioning and Jacobi-PCG on one MI355X.
 *
 * Method (Olenik, Koch, Anzt, "Investigating Matrix Repartitioning to Address
 * the Over- and Undersubscription Challenge for a GPU-based CFD Solver"):
 *  - Sec. 3, repartitioning: GPU part k owns the rows of the alpha CPU ranks
 *    alpha*k .. alpha*k+alpha-1 (blockwise map).  Their LDU sparsity patterns,
 *    including the processor-interface couplings, are fused once into one
 *    row-major (CSR) pattern; couplings whose partner row is now on the same
 *    part are localised, the rest form a non-local block.  The fusion yields
 *    the pattern, the update pattern U (where each rank's coefficients land in
 *    a contiguous receive buffer) and the permutation P (buffer order -> CSR
 *    order).
 *  - Sec. 3, update procedure: pattern and values are separate; every
 *    timestep each rank's coefficients go into the receive buffer, ordered by
 *    originating rank and LDU order, and are reordered by P into the matrix.
 *  - Sec. 4: the pressure system is solved with CG on the GPU; here with a
 *    Jacobi preconditioner, in FP64 or as FP32-inner / FP64-outer iterative
 *    refinement, plus the adjoint (transposed) solve and value gradients.
 *
 * Conventions used by every call:
 *  - Integers are int32 unless stated; every call returns an int status.
 *  - "Device pointer" = memory from hipMalloc on the plan's GPU; "host or
 *    device" = either (resolved through HIP's unified addressing).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued in stream order; calls that must read results on the
 *    host (plan creation, solve, get_*) synchronise that stream themselves.
 *  - No call throws; on failure the status is negative and rp_last_error()
 *    returns a message for the calling thread.
 *  - A plan is not thread-safe; distinct plans are independent.
 *
 * LDU layout (the paper names the LDU host format without defining it):
 *   A(owner[f], neighbour[f]) = upper[f], A(neighbour[f], owner[f]) = lower[f],
 *   A(c, c) = diag[c]; an interface value is the matrix entry A(row, col) of
 *   this rank's row.  Rank r's global rows are [off_r, off_r + n_cells_r),
 *   off_r = sum of n_cells over ranks below r.
 *
 * Receive-buffer ("slot") order, the order of P and of value gradients:
 *   share ranks in order, each as [diag | upper | lower | interface].
 * CSR order: rows ascending, columns ascending within a row.
 */
#ifndef RP_H
#define RP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define RP_OK 0
#define RP_NOT_CONVERGED 1        /* iteration budget spent; x holds the last iterate */
#define RP_ERR_ARG (-1)           /* bad count, null pointer, share outside the ranks */
#define RP_ERR_MESH (-2)          /* addressing out of range, owner == neighbour,
                                     duplicate matrix entry, unpaired interface */
#define RP_ERR_OVERFLOW (-3)      /* rows or slots of the share reach 2^31 */
#define RP_ERR_HIP (-4)           /* a HIP runtime call failed */
#define RP_ERR_UNSUPPORTED (-5)   /* solve with a non-empty non-local block, CG on a
                                     non-symmetric matrix, BiCGStab not in FP64 */
#define RP_ERR_BREAKDOWN (-6)     /* CG: p.Ap <= 0 or not finite; BiCGStab: (rh, r),
                                     (rh, v) or (t, t) zero or not finite, or omega = 0 */
#define RP_ERR_VALUE (-7)         /* an updated value is not finite, or diag <= 0 */

/* ---- precisions -------------------------------------------------------- */
#define RP_FP64 0                 /* FP64 everywhere */
#define RP_MIXED 1                /* mixed-precision iterative refinement (solve only): FP64
                                     residual and solution, FP32 inner PCG to inner_tol */
#define RP_FP32 2                 /* FP32 matrix and vectors (rp_spmv only) */
#define RP_MIXED_RR 3             /* FP32 PCG with FP64 residual replacement every
                                     update_delta reduction (solve only) */

/* ---- preconditioners ---------------------------------------------------- */
#define RP_PRECOND_JACOBI 0       /* M = diag(A) */
#define RP_PRECOND_BLOCK_JACOBI 1 /* M = the diagonal blocks of block_size consecutive rows,
                                     every block inside one CPU rank (CG only) */
#define RP_BJ_MAX_BLOCK 8
#define RP_PRECOND_AMG 2          /* M^-1 = one V-cycle of aggregation multigrid on the
                                     whole system, fused or solve order (CG only;
                                     rp_plan_amg_setup) */
#define RP_AMG_OMEGA 0.8          /* damping of the multigrid's Jacobi sweeps */
#define RP_AMG_COARSE_MAX 64      /* rows of the coarsest level at most (dense inverse) */
#define RP_AMG_TAIL_ROWS 1024     /* the V-cycle from the first level (below the fine one)
                                     with at most this many rows down runs in one workgroup */

/* ---- launches per Jacobi-PCG iteration (rp_solve_opts.fused_loop) ------- */
#define RP_LOOP_AUTO 0            /* two launches on systems of at most RP_LOOP_TWO_MAX_ROWS
                                     rows, three on larger ones */
#define RP_LOOP_COOPERATIVE 1     /* all iterations in one cooperative launch */
#define RP_LOOP_THREE 2           /* three launches (SpMV; r update; x and p update) */
#define RP_LOOP_TWO_MAX_ROWS 262144

/* ---- Krylov methods ------------------------------------------------------ */
#define RP_CG 0                   /* Jacobi-PCG, symmetric positive definite A (the pressure
                                     system, Sec. 4) */
#define RP_BICGSTAB 1             /* Jacobi right-preconditioned BiCGStab, any non-singular A
                                     (the non-symmetric momentum system, Sec. 4); FP64 only */

typedef struct rp_plan rp_plan;

/* One CPU rank's LDU addressing (Sec. 3, step 1: the pattern including the
 * coupling terms to non-local entries).  All arrays are host memory, owned by
 * the caller and only read during rp_plan_create. */
typedef struct rp_rank_desc {
    int32_t n_cells;                 /* rows of this rank */
    int32_t n_faces;                 /* internal faces */
    const int32_t* owner;            /* [n_faces] local cell of the upper entry's row */
    const int32_t* neighbour;        /* [n_faces] local cell of the upper entry's column */
    int32_t n_iface;                 /* processor-interface couplings */
    const int32_t* iface_cell;       /* [n_iface] local cell on this rank (the row) */
    const int32_t* iface_nbr_rank;   /* [n_iface] rank owning the cell across the face */
    const int32_t* iface_nbr_cell;   /* [n_iface] that cell's local id on its rank (the column) */
} rp_rank_desc;

typedef struct rp_solve_opts {
    double tol;              /* stop when ||b - A x||_2 <= tol ||b||_2 (default 1e-8) */
    double inner_tol;        /* RP_MIXED: each inner FP32 PCG stops at this relative
                                residual, or earlier once its residual is below
                                tol ||b|| / 2 (default 1e-4) */
    double update_delta;     /* RP_MIXED_RR: the FP64 update is due once the FP32 residual has
                                fallen by this factor since the last one (default 0.1) */
    int32_t max_iter;        /* FP64: CG iterations; mixed: total FP32 iterations */
    int32_t precision;       /* RP_FP64, RP_MIXED or RP_MIXED_RR */
    int32_t max_outer;       /* mixed: FP64 residual updates / refinement steps (default 200) */
    int32_t check_every;     /* host reads the device convergence state every this
                                many iterations (default 32); iteration counts do
                                not depend on it */
    int32_t x0_zero;         /* 1: start from x = 0 and ignore x on entry */
    int32_t max_restarts;    /* FP64: restarts when the recurrence residual passes
                                but the true residual does not (default 5) */
    int32_t method;          /* RP_CG (default) or RP_BICGSTAB */
    int32_t transpose;       /* 1: solve A^T x = b (the adjoint solve); with RP_CG, where A
                                is symmetric, this is the same system (default 0) */
    int32_t graph;           /* RP_CG, 1: launch each check_every-iteration chunk as one
                                replay of a HIP graph captured on first use and kept in
                                the plan (captured again when a solve's vectors or chunk
                                length differ).  Same arithmetic and results as 0; pays
                                off where launches, not the SpMV, bound an iteration.
                                Ignored while kernel timing is on and by RP_BICGSTAB
                                (default 0) */
    int32_t precond;         /* RP_PRECOND_JACOBI (default), RP_PRECOND_BLOCK_JACOBI or RP_PRECOND_AMG
                                (RP_CG, fused solve order; FP64 and both mixed forms) */
    int32_t block_size;      /* block-Jacobi rows per block, 1..RP_BJ_MAX_BLOCK (default 4) */
    int32_t fused_loop;      /* RP_CG with Jacobi, how an iteration is launched.
                                RP_LOOP_THREE: one launch per phase (SpMV with (p, q);
                                r update with (r, z), (r, r); x and p update).
                                RP_LOOP_AUTO (default): the same on systems above
                                RP_LOOP_TWO_MAX_ROWS rows; on smaller ones two launches, the
                                x and p update of iteration k fused with the SpMV of k + 1
                                (each row forms the new p of its columns itself), with
                                results bit-identical to RP_LOOP_THREE.
                                RP_LOOP_COOPERATIVE: all iterations in one cooperative
                                launch (the phases separated by grid-wide barriers; same
                                arithmetic, partial sums over a smaller grid); on MI355X it
                                measured slower at every size tried, since each barrier
                                writes back and invalidates a die's L2 per block.
                                Kernel timing, graph replay, block-Jacobi and the
                                multigrid always take three launches per iteration, as
                                does RP_LOOP_COOPERATIVE where the device cannot launch
                                the grid cooperatively. */
} rp_solve_opts;

typedef struct rp_solve_info {
    int32_t status;          /* the returned status */
    int32_t iters;           /* FP64 CG iterations, or total FP32 iterations */
    int32_t outer_iters;     /* mixed: FP64 residual updates (0 for RP_FP64) */
    int32_t restarts;        /* true-residual restarts */
    double rel_res;          /* ||b - A x||_2 / ||b||_2 at exit, FP64 on the GPU */
} rp_solve_info;

/* ---- plan (Sec. 3: steps 1-3 and the three resulting structures) ------- *
 * Fuse ranks first_rank .. first_rank+alpha-1 of n_ranks_total CPU ranks.
 * n_cells_all[n_ranks_total]: rows of every rank (host).  share[alpha]: the
 * addressing of the fused ranks.  Builds pattern, U and P on the current HIP
 * device and allocates the matrix and solver workspace there.  Validation:
 * every index in range, owner != neighbour, no matrix entry twice, every
 * interface coupling (c, q, d) on rank p with q in the share matched by
 * (d, p, c) on rank q.  *out receives the plan, or NULL on failure. */
int rp_plan_create(int32_t n_ranks_total, const int32_t* n_cells_all, int32_t first_rank,
                   int32_t alpha, const rp_rank_desc* share, rp_plan** out);

void rp_plan_destroy(rp_plan* plan);

/* Sizes: rows, local and non-local entries, slots (= buffer length).
 * slot_off[alpha+1] (nullable): buffer offset of each share rank's slot block
 * (the update pattern U).  Any output pointer may be NULL. */
int rp_plan_sizes(const rp_plan* plan, int64_t* n_rows, int64_t* nnz_local,
                  int64_t* nnz_nonlocal, int64_t* n_slots, int64_t* slot_off);

/* Copy the fused pattern to caller-allocated host buffers (any may be NULL):
 * row_ptr[n_rows+1], col[nnz_local] (local column ids), perm[n_slots] (P:
 * slot -> CSR position; non-local slots map to nnz_local + their position in
 * the non-local block), nl_row_ptr[n_rows+1], nl_col[nnz_nonlocal] (global
 * column ids, int64). */
int rp_plan_get_csr(rp_plan* plan, int32_t* row_ptr, int32_t* col, int32_t* perm,
                    int32_t* nl_row_ptr, int64_t* nl_col);

/* Device pointers to the plan's pattern and current values, valid until
 * rp_plan_destroy and read-only for the caller.  The arrays keep the layouts
 * of rp_plan_get_csr and rp_plan_get_values; the values change with every
 * update, so read them in stream order after it.  No device work, no sync. */
typedef struct rp_device_ptrs {
    const int32_t* row_ptr;     /* [n_rows+1] fused local block */
    const int32_t* col;         /* [nnz_local] local column ids, ascending per row */
    const int32_t* perm;        /* [n_slots] P: slot -> CSR position */
    const int32_t* nl_row_ptr;  /* [n_rows+1] non-local block */
    const int64_t* nl_col;      /* [nnz_nonlocal] global column ids */
    const double* val64;        /* [n_slots] CSR order, local block then non-local */
    const float* val32;         /* [n_slots] RNE copy of val64 */
    const double* dinv64;       /* [n_rows] 1 / diag */
    const float* dinv32;        /* [n_rows] RNE copy of dinv64 */
    const double* recv;         /* [n_slots] receive buffer, slot order: holds the
                                   values of the last update from host memory
                                   (device-resident rank arrays are read in place) */
} rp_device_ptrs;
int rp_plan_device_ptrs(const rp_plan* plan, rp_device_ptrs* out);

/* Copy the current values to caller-allocated host buffers (any may be NULL):
 * val64[n_slots], val32[n_slots] (CSR order, local block then non-local),
 * dinv64[n_rows] = 1/diag, dinv32[n_rows].  Synchronises the plan. */
int rp_plan_get_values(rp_plan* plan, double* val64, float* val32, double* dinv64,
                       float* dinv32);

/* LDS x windows of the SpMV.  When the plan is built, the share's face
 * offsets give a window layout: *mode = -1 none, 0 a window around the
 * diagonal, 1 or 2: also that many pairs of windows at -d and +d rows,
 * offsets[0..mode) = d.  *enabled says whether the SpMV kernels stage x
 * through those windows (off by default: on MI355X the direct x loads
 * measured faster).  Any output may be NULL.  Results of every kernel are
 * identical either way; only where x is read from changes. */
int rp_plan_spmv_windows(const rp_plan* plan, int32_t* mode, int32_t* offsets, int32_t* enabled);
int rp_plan_set_spmv_windows(rp_plan* plan, int32_t enable);

/* Column-index form of the SpMV.  When the plan is built, every group of 256
 * consecutive fused rows whose entries use at most 16 distinct offsets
 * col - row (a stencil in a rank's natural cell order) is offset-coded: the
 * SpMV kernels keep its CSR values but take the columns from one ascending
 * offset table per group and a 16-bit mask per row instead of reading col;
 * every other group (scrambled numbering, many offsets) is read as CSR.
 * Products and row sums are formed in the same order either way, so every
 * result is identical; only the bytes read change.  bytes64 / bytes32 are
 * the algorithmic HBM bytes of one y = A x in the form in use (each value,
 * index word, x and y element once). */
typedef struct rp_spmv_format {
    int32_t enabled;       /* the kernels use the coded groups (default 1) */
    int32_t reserved;
    int64_t n_groups;      /* groups of 256 rows */
    int64_t coded_groups;  /* groups that are offset-coded */
    int64_t coded_rows;
    int64_t coded_nnz;
    int64_t bytes64;
    int64_t bytes32;
} rp_spmv_format;
int rp_plan_spmv_format(const rp_plan* plan, rp_spmv_format* info);
/* enable = 0: every group as CSR; 1: coded groups where built (default). */
int rp_plan_set_spmv_format(rp_plan* plan, int32_t enable);

/* ---- solve order (an implementation choice; the solvers of Sec. 4 are
 * unchanged, only the numbering they run in) ------------------------------ *
 * mode 0 (default): every rp_solve runs on the fused row order.  mode 1:
 * CG, the mixed solvers and BiCGStab (also transposed) run on a reverse
 * Cuthill-McKee renumbering of the fused local block.  The first call with
 * mode 1 builds it (pattern downloaded, order and renumbered CSR computed on
 * the host, uploaded; synchronises the device).  The renumbered values
 * follow every update through one gather, done by the next solve.  b and x
 * of rp_solve stay in fused order; the solve permutes them in and out.  The
 * pattern, P, rp_update_values*, rp_spmv and rp_value_grad keep the fused
 * order.  Results equal the fused
 * order's up to rounding (each row's products are summed in ascending
 * renumbered column).  Pays off where the fused numbering has no locality
 * (scrambled meshes); on a naturally ordered mesh it replaces the
 * offset-coded SpMV by plain CSR and is slower.  mode 0 or 1, else
 * RP_ERR_ARG; a share with non-local entries: RP_ERR_UNSUPPORTED. */
int rp_plan_set_solve_order(rp_plan* plan, int32_t mode);
/* *mode (nullable): the current mode.  perm[n_rows] (nullable): the fused
 * row at each solve-order position; RP_ERR_ARG if no order was built. */
int rp_plan_solve_order(const rp_plan* plan, int32_t* mode, int32_t* perm);
/* The ordering itself, on host arrays (no device work): reverse
 * Cuthill-McKee of the n x n pattern (row_ptr[n+1] from 0, col[row_ptr[n]]
 * in [0, n), structurally symmetric; diagonal entries ignored).  Each
 * connected component, in order of its lowest row, starts from a
 * pseudo-peripheral row; neighbours are visited by ascending degree, ties by
 * index; the order is then reversed.  perm[k] = the row placed at k.
 * RP_ERR_ARG on a malformed pattern. */
int rp_rcm_order(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* perm);

/* ---- update (Sec. 3, update procedure) --------------------------------- *
 * diag/upper/lower/iface: arrays of alpha pointers (host array), pointer s
 * giving rank first_rank+s's values in its LDU order (host or device memory).
 * lower == NULL means symmetric (lower = upper).  Stages the values into the
 * receive buffer at U's offsets (host memory: per-rank copies; device
 * memory: one staging kernel) and reorders them by P into the FP64 matrix,
 * its FP32 copy (round to nearest even) and the Jacobi inverse diagonal
 * (one IEEE division, then rounded to FP32).  Asynchronous on `stream`: the
 * inputs must stay unchanged until the stream has passed this call.  A value
 * that is not finite or a diagonal <= 0 is recorded on the device and
 * reported as RP_ERR_VALUE by the next rp_sync / rp_solve. */
int rp_update_values(rp_plan* plan, const double* const* diag, const double* const* upper,
                     const double* const* lower, const double* const* iface, void* stream);

/* Same as rp_update_values with the receive buffer already filled by the
 * caller: slots[n_slots] is a device array in slot order (the buffer that
 * ranks write straight into when they can reach device memory). */
int rp_update_values_slots(rp_plan* plan, const double* slots, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * update as rp_update_values with every per-rank array in device memory,
 * same results bit for bit.  Its only scratch, the table of 4 pointers per
 * rank that the reorder reads, lives in a fixed library-owned device array
 * of 4 * RP_NOALLOC_MAX_RANKS pointers (128 KiB on each GPU the library runs
 * on, held until the process ends) instead of plan memory, and the call
 * makes no hipMalloc or hipFree.  RP_ERR_ARG for a share of more than
 * RP_NOALLOC_MAX_RANKS ranks or an array that is not device memory (checked
 * before any device work).  Every call on one GPU shares that array: calls
 * that overlap on one GPU (other streams, threads or plans) race, so the
 * caller serialises them. */
#define RP_NOALLOC_MAX_RANKS 4096
int rp_update_values_noalloc(rp_plan* plan, const double* const* diag, const double* const* upper,
                             const double* const* lower, const double* const* iface, void* stream);

/* ---- ranks in other processes (Sec. 3 update procedure; the GPU-aware
 * communication study of Sec. 4) -------------------------------------------- *
 * The owner exports its plan's receive buffer (device memory, n_slots
 * doubles) as an IPC handle; a rank process attaches it and writes its own
 * slot block [diag | upper | lower | interface] at its offset of U
 * (rp_plan_sizes' slot_off) straight into the owner's device memory, the
 * one-GPU analogue of a rank sending with GPU-aware MPI.  When every rank
 * has returned from rp_recv_write, the owner reorders the buffer with
 * rp_update_values_slots(plan, recv, stream), recv from
 * rp_plan_device_ptrs.  Ranks write disjoint slot ranges; the owner must not
 * update from the buffer while writes are in progress. */
typedef struct rp_ipc_handle {
    char bytes[64];            /* opaque; hipIpcMemHandle_t of the receive buffer */
} rp_ipc_handle;
/* Owner side.  RP_ERR_UNSUPPORTED for a buffer of 2 GiB or more. */
int rp_plan_export_recv(rp_plan* plan, rp_ipc_handle* out, int64_t* n_slots);
/* Rank side (another process, same GPU current): map the owner's buffer;
 * *recv is a device pointer into it, valid until rp_recv_detach. */
int rp_recv_attach(const rp_ipc_handle* handle, double** recv);
/* Copy one rank's values (host or device memory; lower NULL = symmetric, the
 * lower region gets upper) to recv[slot_offset ...] in its LDU order.
 * Returns when the values are in the owner's device memory. */
int rp_recv_write(double* recv, int64_t slot_offset, const double* diag, int32_t n_cells,
                  const double* upper, int32_t n_faces, const double* lower, const double* iface,
                  int32_t n_iface, void* stream);
int rp_recv_detach(double* recv);

/* ---- kernels on the fused matrix ---------------------------------------- *
 * y = A x over the local block, x and y device arrays of n_rows elements:
 * double with RP_FP64, float with RP_FP32.  Each row is summed from 0 in
 * column order with one rounding per product and per sum. */
int rp_spmv(rp_plan* plan, int32_t precision, const void* x, void* y, void* stream);

/* ---- solve (Sec. 4: CG for the pressure system, BiCGStab for momentum) -- *
 * opts->method = RP_CG (default): RP_FP64 is Jacobi-PCG in FP64.  RP_MIXED
 * is iterative refinement: the FP64 residual r = b - A x is rounded to FP32,
 * an FP32 Jacobi-PCG (FP32 matrix, preconditioner, vectors and dot products)
 * solves A d = r from d = 0 until its residual is below inner_tol times its
 * start (or below tol ||b|| / 2, the outer target, if that is reached
 * first), x += d in FP64, and this repeats until the FP64 residual meets tol.
 * RP_MIXED_RR runs one FP32 PCG throughout and, whenever its residual has
 * fallen by update_delta, folds its correction into the FP64 solution and
 * replaces its residual by the FP64 residual b - A x, keeping the search
 * direction; the stop test is on that FP64 residual.
 * opts->method = RP_BICGSTAB: BiCGStab with M = diag(A) applied on the
 * right, in FP64, for non-symmetric matrices (van der Vorst 1992; one
 * iteration = two products with A); its stop test and restart follow the
 * CG's.  opts->transpose = 1 solves A^T x = b: A's values are gathered into
 * A^T's (the fused pattern is structurally symmetric, so every entry (i, j)
 * has a partner (j, i)) whenever they changed since the last such solve.
 * b, x: device arrays of n_rows doubles in fused row order (the share's
 * ranks in order, each in local cell order).  x holds x0 on entry (unless
 * opts->x0_zero) and the solution on return.  opts NULL = defaults.  Blocks
 * until the solve is finished.  Returns RP_OK, RP_NOT_CONVERGED,
 * RP_ERR_BREAKDOWN, RP_ERR_UNSUPPORTED (non-local block, CG on a
 * non-symmetric matrix, BiCGStab not in FP64), RP_ERR_VALUE (a pending update
 * error).  b = 0 gives x = 0. */
int rp_solve(rp_plan* plan, const double* b, double* x, const rp_solve_opts* opts,
             rp_solve_info* info, void* stream);

void rp_solve_opts_default(rp_solve_opts* opts);

/* ---- adjoint -------------------------------------------------------------- *
 * Gradient of a loss L with respect to every receive-buffer slot, given the
 * forward solution x and lambda = A^-T dL/dx (for symmetric A, one more
 * rp_solve): g_slots[k] = -lambda[row(k)] * x[col(k)] (device arrays).  Under
 * the symmetric convention the caller adds the upper and lower slot
 * gradients of a face. */
int rp_value_grad(rp_plan* plan, const double* lambda, const double* x, double* g_slots,
                  void* stream);

/* Block-Jacobi preconditioner (the stronger preconditioner of the outlook in
 * Sec. 5), with every block inside one CPU rank: each share rank's fused
 * rows are cut into runs of block_size consecutive rows (a rank's last run
 * may be shorter), and M = blockdiag(A_bb).  Each diagonal block is inverted
 * by Gauss-Jordan elimination without pivoting (pivots in order; A is SPD),
 * and the upper triangle of the inverse serves both triangles, so M^-1 is
 * exactly symmetric.  Built on the GPU by the first solve that asks for it
 * after each update; this call builds it for the current values (it
 * synchronises) and copies it out (any output may be NULL): n_blocks,
 * start[n_blocks+1] (first fused row of each block), and the packed upper
 * triangles minv64 / minv32 [n_blocks * P], P = bs (bs + 1) / 2, entry
 * (i, j), i <= j < rows of the block, at b * P + i bs - i (i - 1) / 2 + j - i
 * (unused entries 0; minv32 = RNE(minv64)).  RP_ERR_BREAKDOWN when a block
 * is not positive definite. */
int rp_plan_block_jacobi(rp_plan* plan, int32_t block_size, int64_t* n_blocks, int32_t* start,
                         double* minv64, float* minv32);

/* Aggregation multigrid preconditioner (the multigrid option of the outlook
 * in Sec. 5) over the plan's whole fused system; needs an empty non-local
 * block and, like CG, a symmetric matrix.
 *
 * Hierarchy.  Level 0 is the fused local block.  Level l (n rows) is the
 * coarsest when n <= RP_AMG_COARSE_MAX; otherwise:
 *  1. strength of an entry (i, j), j != i, with value a < 0: the key
 *     (-a, h, min(i,j), max(i,j)), h = fmix32(min * 0x9E3779B1 + max mod 2^32)
 *     (MurmurHash3's 32-bit finaliser); larger -a is stronger, then larger
 *     h, then the smaller (min, max).  Entries with a >= 0 never couple.
 *  2. matching rounds (at most 16, until a round forms no pair): every
 *     unmatched row picks its strongest coupling to an unmatched row; rows
 *     that picked each other pair up.
 *  3. a row left unmatched joins the pair of its strongest coupling to a
 *     matched row, else stays alone.  Aggregates (a pair with its joiners,
 *     or a lone row) are numbered by their leaders (a pair's smaller row)
 *     ascending: agg[i] is row i's coarse row.  No aggregate formed at all
 *     is RP_ERR_UNSUPPORTED.
 *  4. A_c = P^T A P (P[i][agg[i]] = 1): each coarse entry sums its fine
 *     entries from 0 in ascending fine CSR position; columns ascending;
 *     dinv = 1 / diagonal.
 *  5. the coarsest matrix is inverted densely by Gauss-Jordan without
 *     pivoting (RP_ERR_BREAKDOWN if a pivot or coarse diagonal is not > 0).
 * V-cycle y = V_l(r): coarsest y = A_L^-1 r (row sums in column order);
 * even l: x = omega (dinv r), t = r - A x, r'_I = sum of t over aggregate
 * I's rows ascending, x += V_{l+1}(r')[agg], y = x + omega (dinv (r - A x));
 * odd l: r'_I = sum of r over the members, y = V_{l+1}(r')[agg];
 * omega = RP_AMG_OMEGA.  Row sums of A x in column order from 0.  The FP32
 * inner solves use the same hierarchy with every value rounded to FP32.
 *
 * The first solve with RP_PRECOND_AMG builds the hierarchy from the values at
 * hand; later value updates keep the aggregates and patterns and refresh the
 * coarse values (steps 4-5) at the next such solve.  With the solve order
 * (rp_plan_set_solve_order) the plan keeps a second hierarchy, built the
 * same way on the renumbered system.  rp_plan_amg_setup rebuilds the fused
 * hierarchy from the current values and drops the solve-order one, which
 * the next multigrid solve in solve order rebuilds (synchronises on
 * stream). */
int rp_plan_amg_setup(rp_plan* plan, void* stream);

/* Number of levels of the hierarchy (0 before the first setup). */
int rp_plan_amg_levels(const rp_plan* plan, int32_t* n_levels);

/* Host copies of level l (values current for the last refresh; synchronises):
 * n, nnz, row_ptr[n+1], col[nnz], val[nnz] (FP64), dinv[n], and, on all
 * levels but the coarsest, agg[n], mem_ptr[n_{l+1}+1], mem[n] (the rows of
 * each aggregate, ascending).  Any output pointer may be NULL.
 * RP_ERR_ARG for a level outside 0..n_levels-1. */
int rp_plan_amg_level(const rp_plan* plan, int32_t level, int64_t* n, int64_t* nnz, int32_t* row_ptr, int32_t* col,
                      double* val, double* dinv, int32_t* agg, int32_t* mem_ptr, int32_t* mem);

/* Host copy of the coarsest level's dense inverse, row-major [n_L * n_L]. */
int rp_plan_amg_coarse_inverse(const rp_plan* plan, double* cinv);

/* z = V_0(r) in FP64 for device vectors r, z of n_rows (fused order), with
 * the hierarchy current for the plan's values (built or refreshed first);
 * enqueued on stream. */
int rp_plan_amg_apply(rp_plan* plan, const double* r, double* z, void* stream);

/* Launch shape of the solvers' elementwise kernels (a diagnostic knob; the
 * default sizes the grid to n_rows, at most 1024 blocks).  blocks = 0 restores
 * the default; 1..16384 fixes the grid, far beyond what the chip holds at
 * once, so that blocks of one launch start after others have finished.
 * Results are the same for any grid except for the rounding of dot products
 * (one partial sum per block).  RP_ERR_ARG outside 0..16384. */
int rp_plan_set_vec_grid(rp_plan* plan, int32_t blocks);

/* ---- lifetime / diagnostics --------------------------------------------- */
/* Wait for the plan's pending work; reports a pending RP_ERR_VALUE. */
int rp_sync(rp_plan* plan);

/* Message of the calling thread's last failure ("" if none). */
const char* rp_last_error(void);

/* Kernel timing with HIP events on the launch stream (off by default).  While
 * enabled, every enable-th launch of kernel `kernel` (RP_KERNEL_*) is
 * bracketed by an event pair (enable = 1: every launch; an event pair costs
 * the stream several microseconds, so a stride above 1 keeps the timed run
 * close to an untimed one); rp_plan_kernel_stats returns the count of the
 * recorded launches that did work and their summed device time since
 * enabling.  enable = 0 switches timing off; below 0 is an argument error. */
#define RP_KERNEL_SPMV64 0        /* FP64 CSR SpMV inside CG (q = A p with p.q) */
#define RP_KERNEL_SPMV32 1        /* FP32 CSR SpMV inside the inner CG */
#define RP_KERNEL_SCATTER 2       /* value update (reorder by P) */
#define RP_N_KERNELS 3
int rp_plan_set_timing(rp_plan* plan, int32_t enable);
int rp_plan_kernel_stats(rp_plan* plan, int32_t kernel, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* RP_H */

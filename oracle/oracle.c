/*
 * Serial FP64 oracle for the matrix-repartitioning path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU definition of what the GPU library computes.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it; the product
 * library neither links nor calls it, and the two share no code.
 *
 * Built with gcc -O2 -ffp-contract=off (no fused multiply-add, no fast-math):
 * every product and sum below is one correctly rounded IEEE operation, taken
 * in the order written.
 *
 * Paper: Olenik, Koch, Anzt, "Investigating Matrix Repartitioning to Address
 * the Over- and Undersubscription Challenge for a GPU-based CFD Solver".
 *
 * Readings of the paper used here (the paper leaves these open):
 *  - LDU layout (Sec. 3 names the LDU host format without defining it):
 *    A(owner_f, neighbour_f) = upper[f], A(neighbour_f, owner_f) = lower[f],
 *    A(c, c) = diag[c]; interface value = the matrix entry A(row, col).
 *  - Global row ids of CPU rank r (the index sets I_CPU(r) of Sec. 3) are the
 *    contiguous range [off_r, off_r + n_cells_r), off_r = sum of n_cells over
 *    ranks below r; the GPU part k then owns one contiguous range.
 *  - Receive-buffer order (Sec. 3, update procedure): ranks of the share in
 *    order; inside a rank [diag | upper | lower | interface], each in the
 *    rank's own LDU order.
 *  - Device order (Sec. 3, "row-major"): rows ascending, columns ascending
 *    within a row; the local block first, then the non-local block.
 *  - Preconditioner: Jacobi, M = diag(A) (the paper only names CG, Sec. 4).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_ERR_ARG (-1)
#define OR_ERR_MESH (-2)
#define OR_ERR_OVERFLOW (-3)
#define OR_ERR_BREAKDOWN (-6)

/* ------------------------------------------------------------------------ *
 * Sizes of the merged system for the share [first, first + alpha).
 * ------------------------------------------------------------------------ */
int or_merge_sizes(int alpha, const int32_t* n_cells_share, const int32_t* n_faces,
                   const int32_t* n_iface, int64_t* n_rows, int64_t* n_slots)
{
    int64_t rows = 0, slots = 0;
    for (int s = 0; s < alpha; ++s) {
        rows += n_cells_share[s];
        slots += (int64_t)n_cells_share[s] + 2 * (int64_t)n_faces[s] + n_iface[s];
    }
    *n_rows = rows;
    *n_slots = slots;
    return OR_OK;
}

/* ------------------------------------------------------------------------ *
 * Repartition (Sec. 3, steps 1-3 and the three resulting structures).
 *
 * GPU part k fuses the patterns of CPU ranks first..first+alpha-1 (the
 * blockwise map of Sec. 3).  Every LDU coefficient of those ranks is one
 * "slot" of the contiguous receive buffer; the slot's matrix position is
 *   diag  c   -> (off_r + c,      off_r + c)
 *   upper f   -> (off_r + own_f,  off_r + nbr_f)
 *   lower f   -> (off_r + nbr_f,  off_r + own_f)
 *   iface e   -> (off_r + cell_e, off_q + ncell_e),  q = nbr rank of e
 * A slot is local when its global column lies in the fused row set
 * I_GPU = union of I_CPU(r) over the share (the localisation rule of Sec. 3),
 * non-local otherwise.  Rows are numbered from the start of the share.
 *
 * Outputs (caller allocated):
 *   row_ptr[n_rows+1], col[n_slots] (local column ids; first nnz_local used)
 *   nl_row_ptr[n_rows+1], nl_col[n_slots] (global column ids)
 *   perm[n_slots]: slot -> device position (local block 0..nnz_local-1, then
 *                  the non-local block nnz_local + position); the permutation
 *                  P of Sec. 3
 *   slot_off[alpha+1]: receive-buffer offset of each rank's slot block; with
 *                  the lengths this is the update pattern U of Sec. 3
 *   slot_row[n_slots], slot_col[n_slots]: matrix position of every slot
 *                  (row from the share start, column global)
 *   diag_slot[n_rows]: the slot holding each row's diagonal
 *   counts[2] = {nnz_local, nnz_nonlocal}
 * ------------------------------------------------------------------------ */
int or_merge(int n_ranks_total, const int32_t* n_cells_all, int first, int alpha,
             const int32_t* n_faces, const int32_t* owner, const int32_t* neighbour,
             const int32_t* n_iface, const int32_t* iface_cell,
             const int32_t* iface_nbr_rank, const int32_t* iface_nbr_cell,
             int32_t* row_ptr, int32_t* col, int32_t* nl_row_ptr, int64_t* nl_col,
             int32_t* perm, int64_t* slot_off, int32_t* slot_row, int64_t* slot_col,
             int32_t* diag_slot, int64_t* counts)
{
    if (n_ranks_total < 1 || alpha < 1 || first < 0 || first + alpha > n_ranks_total)
        return OR_ERR_ARG;

    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (n_ranks_total + 1));
    off[0] = 0;
    for (int r = 0; r < n_ranks_total; ++r) {
        if (n_cells_all[r] < 0) { free(off); return OR_ERR_ARG; }
        off[r + 1] = off[r] + n_cells_all[r];
    }
    const int64_t lo = off[first], hi = off[first + alpha];
    const int64_t n_rows = hi - lo;

    /* slot coordinates, in buffer order */
    int64_t k = 0, fbase = 0, ebase = 0;
    for (int s = 0; s < alpha; ++s) {
        const int r = first + s;
        const int64_t nc = n_cells_all[r];
        const int64_t row0 = off[r] - lo;
        slot_off[s] = k;
        for (int64_t c = 0; c < nc; ++c) {
            slot_row[k] = (int32_t)(row0 + c);
            slot_col[k] = off[r] + c;
            diag_slot[row0 + c] = (int32_t)k;
            ++k;
        }
        for (int64_t f = 0; f < n_faces[s]; ++f) {
            int32_t o = owner[fbase + f], b = neighbour[fbase + f];
            if (o < 0 || o >= nc || b < 0 || b >= nc || o == b) { free(off); return OR_ERR_MESH; }
            slot_row[k] = (int32_t)(row0 + o);
            slot_col[k] = off[r] + b;
            ++k;
        }
        for (int64_t f = 0; f < n_faces[s]; ++f) {
            int32_t o = owner[fbase + f], b = neighbour[fbase + f];
            slot_row[k] = (int32_t)(row0 + b);
            slot_col[k] = off[r] + o;
            ++k;
        }
        for (int64_t e = 0; e < n_iface[s]; ++e) {
            int32_t c = iface_cell[ebase + e], q = iface_nbr_rank[ebase + e], d = iface_nbr_cell[ebase + e];
            if (c < 0 || c >= nc || q < 0 || q >= n_ranks_total || q == r || d < 0 || d >= n_cells_all[q]) {
                free(off);
                return OR_ERR_MESH;
            }
            slot_row[k] = (int32_t)(row0 + c);
            slot_col[k] = off[q] + d;
            ++k;
        }
        fbase += n_faces[s];
        ebase += n_iface[s];
    }
    slot_off[alpha] = k;
    const int64_t n_slots = k;
    if (n_slots >= INT32_MAX || n_rows >= INT32_MAX) { free(off); return OR_ERR_OVERFLOW; }

    /* count entries per row, local and non-local separately */
    memset(row_ptr, 0, sizeof(int32_t) * (n_rows + 1));
    memset(nl_row_ptr, 0, sizeof(int32_t) * (n_rows + 1));
    for (int64_t j = 0; j < n_slots; ++j) {
        int is_local = slot_col[j] >= lo && slot_col[j] < hi;
        if (is_local) row_ptr[slot_row[j] + 1]++;
        else nl_row_ptr[slot_row[j] + 1]++;
    }
    for (int64_t i = 0; i < n_rows; ++i) {
        row_ptr[i + 1] += row_ptr[i];
        nl_row_ptr[i + 1] += nl_row_ptr[i];
    }
    const int64_t nnz_local = row_ptr[n_rows], nnz_nl = nl_row_ptr[n_rows];

    /* place each slot into its row, keeping every row sorted by column
     * (insertion into the row as slots arrive in buffer order) */
    int32_t* fill = (int32_t*)calloc((size_t)n_rows, sizeof(int32_t));
    int32_t* nl_fill = (int32_t*)calloc((size_t)n_rows, sizeof(int32_t));
    int32_t* at_slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz_local > 0 ? nnz_local : 1));
    int32_t* nl_at_slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz_nl > 0 ? nnz_nl : 1));
    int status = OR_OK;
    for (int64_t j = 0; j < n_slots && status == OR_OK; ++j) {
        const int64_t i = slot_row[j];
        const int64_t cg = slot_col[j];
        const int is_local = cg >= lo && cg < hi;
        const int32_t* rp = is_local ? row_ptr : nl_row_ptr;
        int32_t* fl = is_local ? fill : nl_fill;
        int32_t* at = is_local ? at_slot : nl_at_slot;
        int64_t base = rp[i];
        int64_t m = fl[i];
        /* shift larger columns right, then drop the slot in */
        while (m > 0 && slot_col[at[base + m - 1]] > cg) {
            at[base + m] = at[base + m - 1];
            --m;
        }
        if (m > 0 && slot_col[at[base + m - 1]] == cg) status = OR_ERR_MESH; /* duplicate entry */
        at[base + m] = (int32_t)j;
        fl[i]++;
    }
    if (status == OR_OK) {
        for (int64_t p = 0; p < nnz_local; ++p) {
            col[p] = (int32_t)(slot_col[at_slot[p]] - lo);
            perm[at_slot[p]] = (int32_t)p;
        }
        for (int64_t p = 0; p < nnz_nl; ++p) {
            nl_col[p] = slot_col[nl_at_slot[p]];
            perm[nl_at_slot[p]] = (int32_t)(nnz_local + p);
        }
        /* interface pairing inside the share: the coupling (c, q, d) on rank p
         * needs its partner (d, p, c) on rank q, i.e. an interface slot of q at
         * the transposed position */
        fbase = 0;
        for (int s = 0; s < alpha && status == OR_OK; ++s) {
            const int r = first + s;
            const int64_t e0 = slot_off[s] + n_cells_all[r] + 2 * (int64_t)n_faces[s];
            for (int64_t j = e0; j < slot_off[s + 1]; ++j) {
                const int64_t cg = slot_col[j];
                if (!(cg >= lo && cg < hi)) continue;
                const int64_t prow = cg - lo;                /* partner's row */
                const int64_t want = slot_row[j] + lo;       /* partner's column */
                int found = 0;
                for (int64_t p = row_ptr[prow]; p < row_ptr[prow + 1]; ++p) {
                    if (slot_col[at_slot[p]] == want) {
                        int64_t js = at_slot[p];
                        /* js must be an interface slot of the partner rank */
                        int qs = 0;
                        while (qs < alpha && !(js >= slot_off[qs] && js < slot_off[qs + 1])) ++qs;
                        int64_t qe0 = slot_off[qs] + n_cells_all[first + qs] + 2 * (int64_t)n_faces[qs];
                        found = (js >= qe0);
                        break;
                    }
                }
                if (!found) { status = OR_ERR_MESH; break; }
            }
        }
    }
    counts[0] = nnz_local;
    counts[1] = nnz_nl;
    free(fill); free(nl_fill); free(at_slot); free(nl_at_slot); free(off);
    return status;
}

/* ------------------------------------------------------------------------ *
 * Coefficient update (Sec. 3, update procedure): the receive buffer, ordered
 * by originating rank and LDU order, is reordered by P into the device value
 * array.  FP32 copies are round-to-nearest-even casts; the Jacobi inverse is
 * one correctly rounded FP64 division, then cast.
 * ------------------------------------------------------------------------ */
void or_update(int64_t n_rows, int64_t n_slots, const int32_t* perm, const int32_t* diag_slot,
               const double* buf, double* val64, float* val32, double* dinv64, float* dinv32)
{
    for (int64_t k = 0; k < n_slots; ++k) val64[perm[k]] = buf[k];
    for (int64_t p = 0; p < n_slots; ++p) val32[p] = (float)val64[p];
    for (int64_t i = 0; i < n_rows; ++i) {
        dinv64[i] = 1.0 / buf[diag_slot[i]];
        dinv32[i] = (float)dinv64[i];
    }
}

/* y = A x over the local block: each row summed from 0.0 in column order */
void or_spmv(int64_t n_rows, const int32_t* row_ptr, const int32_t* col, const double* val,
             const double* x, double* y)
{
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) s += val[p] * x[col[p]];
        y[i] = s;
    }
}

static double dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* ‖b − A x‖₂ / ‖b‖₂ (0 when b = 0 and x = 0) */
double or_true_relres(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                      const double* b, const double* x)
{
    double* y = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    or_spmv(n, row_ptr, col, val, x, y);
    double rr = 0.0, bb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = b[i] - y[i];
        rr += d * d;
        bb += b[i] * b[i];
    }
    free(y);
    if (bb == 0.0) return sqrt(rr);
    return sqrt(rr) / sqrt(bb);
}

/* ------------------------------------------------------------------------ *
 * Jacobi-preconditioned conjugate gradients (the CG of Sec. 4 with
 * M = diag(A)), in the textbook order of preconditioned CG:
 *   r = b − A x, z = M⁻¹ r, p = z
 *   repeat: q = A p; a = (r,z)/(q,p); x += a p; r −= a q;
 *           stop if ‖r‖ ≤ tol ‖b‖;
 *           z = M⁻¹ r; beta = (r,z)_new/(r,z)_old; p = z + beta p
 * When the recurrence residual passes, the true residual ‖b − A x‖ is checked;
 * if it fails, CG restarts from the current x (at most max_restarts times).
 * b = 0 gives x = 0 with no iteration.
 * out[0] = iterations, out[1] = restarts; res[0] = true rel. residual.
 * ------------------------------------------------------------------------ */
int or_pcg(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
           const double* b, double* x, double tol, int64_t max_iter, int max_restarts,
           int64_t* out, double* res)
{
    double* diag = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* r = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* z = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* p = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* q = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int status = OR_NOT_CONVERGED;
    int64_t it = 0;
    int restarts = 0;

    for (int64_t i = 0; i < n; ++i) {
        diag[i] = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i) diag[i] = val[k];
    }
    const double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        status = OR_OK;
        goto done;
    }
    for (;;) {
        or_spmv(n, row_ptr, col, val, x, q);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        if (sqrt(dot(n, r, r)) <= tol * bnorm) { status = OR_OK; break; }
        for (int64_t i = 0; i < n; ++i) z[i] = r[i] / diag[i];
        for (int64_t i = 0; i < n; ++i) p[i] = z[i];
        double rz = dot(n, r, z);
        int passed = 0;
        while (it < max_iter) {
            or_spmv(n, row_ptr, col, val, p, q);
            const double pq = dot(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { status = OR_ERR_BREAKDOWN; goto done; }
            const double a = rz / pq;
            for (int64_t i = 0; i < n; ++i) x[i] += a * p[i];
            for (int64_t i = 0; i < n; ++i) r[i] -= a * q[i];
            ++it;
            if (sqrt(dot(n, r, r)) <= tol * bnorm) { passed = 1; break; }
            for (int64_t i = 0; i < n; ++i) z[i] = r[i] / diag[i];
            const double rz_new = dot(n, r, z);
            const double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
        if (!passed) break;                     /* iteration budget spent */
        if (or_true_relres(n, row_ptr, col, val, b, x) <= tol) { status = OR_OK; break; }
        if (restarts >= max_restarts) break;
        ++restarts;
    }
done:
    out[0] = it;
    out[1] = restarts;
    res[0] = or_true_relres(n, row_ptr, col, val, b, x);
    free(diag); free(r); free(z); free(p); free(q);
    return status;
}

/* BiCGStab with Jacobi right preconditioning, M = diag(A): the Krylov
 * solver the paper's benchmark uses for the non-symmetric momentum system
 * (Sec. 4), in the stabilised form of van der Vorst (SIAM J. Sci. Stat.
 * Comput. 13, 1992), as Saad, Iterative Methods for Sparse Linear Systems,
 * 2nd ed., Alg. 7.7, with the preconditioner applied on the right
 * (A M^-1 u = b, x = M^-1 u):
 *   r = b - A x, rh = r, rho0 = alpha = omega = 1, v = p = 0
 *   repeat:  rho = (rh, r);  beta = (rho / rho0) (alpha / omega)
 *            p = r + beta (p - omega v);  y = M^-1 p;  v = A y
 *            alpha = rho / (rh, v);  s = r - alpha v
 *            if ||s|| <= tol ||b||:  x = x + alpha y, stop
 *            z = M^-1 s;  t = A z;  omega = (t, s) / (t, t)
 *            x = (x + alpha y) + omega z;  r = s - omega t;  rho0 = rho
 *            if ||r|| <= tol ||b||: stop
 * One iteration is one pass (two products with A).  A stop on the recurrence
 * residual is confirmed on b - A x; if that fails the method restarts from
 * the current x with rh = r (at most max_restarts times).  rho, (rh, v) or
 * (t, t) equal to 0 or not finite, or omega = 0, is a breakdown.
 * out[0] = iterations, out[1] = restarts; res[0] = true relative residual. */
int or_bicgstab(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                const double* b, double* x, double tol, int64_t max_iter, int max_restarts,
                int64_t* out, double* res)
{
    const size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *diag = (double*)malloc(sz), *r = (double*)malloc(sz), *rh = (double*)malloc(sz);
    double *p = (double*)malloc(sz), *v = (double*)malloc(sz), *y = (double*)malloc(sz);
    double *s = (double*)malloc(sz), *z = (double*)malloc(sz), *t = (double*)malloc(sz);
    int status = OR_NOT_CONVERGED;
    int64_t it = 0;
    int restarts = 0;

    for (int64_t i = 0; i < n; ++i) {
        diag[i] = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i) diag[i] = val[k];
    }
    const double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        status = OR_OK;
        goto done;
    }
    for (;;) {
        or_spmv(n, row_ptr, col, val, x, t);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
        if (sqrt(dot(n, r, r)) <= tol * bnorm) { status = OR_OK; break; }
        for (int64_t i = 0; i < n; ++i) { rh[i] = r[i]; p[i] = 0.0; v[i] = 0.0; }
        double rho0 = 1.0, alpha = 1.0, omega = 1.0;
        int passed = 0;
        while (it < max_iter) {
            const double rho = dot(n, rh, r);
            if (rho == 0.0 || !isfinite(rho)) { status = OR_ERR_BREAKDOWN; goto done; }
            const double beta = (rho / rho0) * (alpha / omega);
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            for (int64_t i = 0; i < n; ++i) y[i] = p[i] / diag[i];
            or_spmv(n, row_ptr, col, val, y, v);
            const double rv = dot(n, rh, v);
            if (rv == 0.0 || !isfinite(rv)) { status = OR_ERR_BREAKDOWN; goto done; }
            alpha = rho / rv;
            for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
            ++it;
            if (sqrt(dot(n, s, s)) <= tol * bnorm) {
                for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * y[i];
                passed = 1;
                break;
            }
            for (int64_t i = 0; i < n; ++i) z[i] = s[i] / diag[i];
            or_spmv(n, row_ptr, col, val, z, t);
            const double tt = dot(n, t, t);
            if (tt == 0.0 || !isfinite(tt)) { status = OR_ERR_BREAKDOWN; goto done; }
            omega = dot(n, t, s) / tt;
            for (int64_t i = 0; i < n; ++i) x[i] = (x[i] + alpha * y[i]) + omega * z[i];
            for (int64_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
            rho0 = rho;
            if (sqrt(dot(n, r, r)) <= tol * bnorm) { passed = 1; break; }
            if (omega == 0.0) { status = OR_ERR_BREAKDOWN; goto done; }
        }
        if (!passed) break;                     /* iteration budget spent */
        if (or_true_relres(n, row_ptr, col, val, b, x) <= tol) { status = OR_OK; break; }
        if (restarts >= max_restarts) break;
        ++restarts;
    }
done:
    out[0] = it;
    out[1] = restarts;
    res[0] = or_true_relres(n, row_ptr, col, val, b, x);
    free(diag); free(r); free(rh); free(p); free(v); free(y); free(s); free(z); free(t);
    return status;
}

/* Gradient of L with respect to every receive-buffer slot for A x = b:
 * dL/dv_k = −lambda_row(k) · x_col(k), lambda = A^-T dL/dx.  Columns are
 * global ids; only local slots (column inside [lo, lo + n_rows)) are defined,
 * non-local slots get 0. */
void or_value_grad(int64_t n_slots, const int32_t* slot_row, const int64_t* slot_col, int64_t lo,
                   int64_t n_rows, const double* lambda, const double* x, double* g)
{
    for (int64_t k = 0; k < n_slots; ++k) {
        const int64_t c = slot_col[k] - lo;
        g[k] = (c >= 0 && c < n_rows) ? -lambda[slot_row[k]] * x[c] : 0.0;
    }
}

/* Gradient with respect to face coefficients c_f of
 * A = sum_f c_f (e_a − e_b)(e_a − e_b)^T + sum_walls c_w e_a e_a^T:
 * interior face: −(lambda_a − lambda_b)(x_a − x_b); wall (b < 0): −lambda_a x_a. */
void or_face_grad(int64_t n_faces, const int64_t* row_a, const int64_t* row_b,
                  const double* lambda, const double* x, double* g)
{
    for (int64_t f = 0; f < n_faces; ++f) {
        const int64_t a = row_a[f], b = row_b[f];
        if (b >= 0) g[f] = -(lambda[a] - lambda[b]) * (x[a] - x[b]);
        else g[f] = -lambda[a] * x[a];
    }
}

/* ------------------------------------------------------------------------ *
 * Block-Jacobi preconditioner: the stronger preconditioner the outlook of
 * Sec. 5 asks for, with every block inside one CPU rank.
 *
 * Blocks: each share rank's rows, in fused order, cut into runs of bs
 * consecutive rows (the last run of a rank may be shorter).  start[b] is the
 * first fused row of block b, start[n_blocks] = n_rows.
 *
 * M = blockdiag(A_bb), A_bb = the entries of the block's rows whose columns
 * lie in the same row range.  Each A_bb is inverted by Gauss-Jordan
 * elimination without pivoting (A is SPD, so are its diagonal blocks, and
 * every pivot is positive), in the textbook order on [W | Z], W = A_bb,
 * Z = I:  for k = 0 .. m-1:  divide row k of W and Z by the pivot W[k][k];
 * then for every row i != k, in ascending order, subtract W[i][k] times row
 * k from row i of W and of Z.  Z is then A_bb^-1.  The preconditioner keeps
 * the upper triangle of Z (i <= j) for both triangles, so M^-1 is exactly
 * symmetric.  Storage: minv[b * P + i * bs - i * (i - 1) / 2 + (j - i)],
 * P = bs (bs + 1) / 2, for 0 <= i <= j < m (unused entries 0).
 * ------------------------------------------------------------------------ */
int64_t or_block_starts(int alpha, const int32_t* n_cells_share, int bs, int32_t* start)
{
    int64_t nb = 0, row = 0;
    for (int s = 0; s < alpha; ++s) {
        for (int64_t c = 0; c < n_cells_share[s]; c += bs) {
            if (start) start[nb] = (int32_t)(row + c);
            ++nb;
        }
        row += n_cells_share[s];
    }
    if (start) start[nb] = (int32_t)row;
    return nb;
}

#define OR_BJ_MAX 8

int or_block_jacobi_inverse(const int32_t* row_ptr, const int32_t* col, const double* val,
                            int64_t n_blocks, const int32_t* start, int bs, double* minv)
{
    if (bs < 1 || bs > OR_BJ_MAX) return OR_ERR_ARG;
    const int64_t P = (int64_t)bs * (bs + 1) / 2;
    for (int64_t b = 0; b < n_blocks; ++b) {
        const int64_t s0 = start[b];
        const int m = (int)(start[b + 1] - s0);
        double W[OR_BJ_MAX][OR_BJ_MAX], Z[OR_BJ_MAX][OR_BJ_MAX];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                W[i][j] = 0.0;
                Z[i][j] = (i == j) ? 1.0 : 0.0;
            }
        for (int i = 0; i < m; ++i)
            for (int64_t p = row_ptr[s0 + i]; p < row_ptr[s0 + i + 1]; ++p) {
                const int64_t c = col[p];
                if (c >= s0 && c < s0 + m) W[i][c - s0] = val[p];
            }
        for (int k = 0; k < m; ++k) {
            const double piv = W[k][k];
            if (!(piv > 0.0) || !isfinite(piv)) return OR_ERR_BREAKDOWN;
            for (int j = 0; j < m; ++j) {
                W[k][j] = W[k][j] / piv;
                Z[k][j] = Z[k][j] / piv;
            }
            for (int i = 0; i < m; ++i) {
                if (i == k) continue;
                const double f = W[i][k];
                for (int j = 0; j < m; ++j) {
                    W[i][j] = W[i][j] - f * W[k][j];
                    Z[i][j] = Z[i][j] - f * Z[k][j];
                }
            }
        }
        double* out = minv + b * P;
        for (int64_t q = 0; q < P; ++q) out[q] = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = i; j < m; ++j) out[i * bs - i * (i - 1) / 2 + (j - i)] = Z[i][j];
    }
    return OR_OK;
}

/* z = M^-1 r: z_i = sum over the block's j ascending of minv(min(i,j), max(i,j)) r_j, from 0 */
void or_block_jacobi_apply(int64_t n_blocks, const int32_t* start, int bs, const double* minv,
                           const double* r, double* z)
{
    const int64_t P = (int64_t)bs * (bs + 1) / 2;
    for (int64_t b = 0; b < n_blocks; ++b) {
        const int64_t s0 = start[b];
        const int m = (int)(start[b + 1] - s0);
        const double* mb = minv + b * P;
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) {
                const int a = i < j ? i : j, c = i < j ? j : i;
                s += mb[a * bs - a * (a - 1) / 2 + (c - a)] * r[s0 + j];
            }
            z[s0 + i] = s;
        }
    }
}

/* PCG exactly as or_pcg, with z = M^-1 r by the block-Jacobi preconditioner
 * of block size bs (blocks from or_block_starts over n_cells_share[alpha]).
 * OR_ERR_BREAKDOWN also for a block that is not positive definite. */
int or_pcg_block_jacobi(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                        int alpha, const int32_t* n_cells_share, int bs,
                        const double* b, double* x, double tol, int64_t max_iter, int max_restarts,
                        int64_t* out, double* res)
{
    const int64_t nb = or_block_starts(alpha, n_cells_share, bs, NULL);
    int32_t* start = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb + 1));
    double* minv = (double*)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1) * (size_t)(bs * (bs + 1) / 2));
    double* r = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* z = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* p = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* q = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int status = OR_NOT_CONVERGED;
    int64_t it = 0;
    int restarts = 0;

    or_block_starts(alpha, n_cells_share, bs, start);
    if (or_block_jacobi_inverse(row_ptr, col, val, nb, start, bs, minv) != OR_OK) {
        status = OR_ERR_BREAKDOWN;
        goto done;
    }
    const double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        status = OR_OK;
        goto done;
    }
    for (;;) {
        or_spmv(n, row_ptr, col, val, x, q);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        if (sqrt(dot(n, r, r)) <= tol * bnorm) { status = OR_OK; break; }
        or_block_jacobi_apply(nb, start, bs, minv, r, z);
        for (int64_t i = 0; i < n; ++i) p[i] = z[i];
        double rz = dot(n, r, z);
        int passed = 0;
        while (it < max_iter) {
            or_spmv(n, row_ptr, col, val, p, q);
            const double pq = dot(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { status = OR_ERR_BREAKDOWN; goto done; }
            const double a = rz / pq;
            for (int64_t i = 0; i < n; ++i) x[i] += a * p[i];
            for (int64_t i = 0; i < n; ++i) r[i] -= a * q[i];
            ++it;
            if (sqrt(dot(n, r, r)) <= tol * bnorm) { passed = 1; break; }
            or_block_jacobi_apply(nb, start, bs, minv, r, z);
            const double rz_new = dot(n, r, z);
            const double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
        if (!passed) break;                     /* iteration budget spent */
        if (or_true_relres(n, row_ptr, col, val, b, x) <= tol) { status = OR_OK; break; }
        if (restarts >= max_restarts) break;
        ++restarts;
    }
done:
    out[0] = it;
    out[1] = restarts;
    res[0] = or_true_relres(n, row_ptr, col, val, b, x);
    free(start); free(minv); free(r); free(z); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ *
 * Aggregation multigrid preconditioner (the multigrid option of the outlook
 * in Sec. 5): unsmoothed aggregation by pairwise matching, Galerkin coarse
 * matrices, one damped-Jacobi sweep before and after the coarse correction
 * on every other level, a dense inverse on the coarsest level.
 *
 * Level 0 is the fused local block.  Level l + 1 is built from level l
 * (n rows, CSR with ascending columns, symmetric, every row holding its
 * diagonal) unless n <= coarse_max, which makes level l the coarsest:
 *
 *  1. Coupling strength of the entry (i, j), j != i, with value a < 0:
 *     key (w, h, lo, hi) with w = -a, lo = min(i, j), hi = max(i, j),
 *     h = fmix32(lo * 0x9E3779B1 + hi mod 2^32) (the 32-bit finaliser of
 *     MurmurHash3, used only to break ties between equal w).  Entry e1 is
 *     stronger than e2 when w1 > w2, or w equal and h1 > h2, or w and h
 *     equal and (lo1, hi1) < (lo2, hi2).  Entries with a >= 0 never couple.
 *  2. Pairwise matching in rounds (at most OR_AMG_ROUNDS): every unmatched
 *     row picks its strongest coupling to an unmatched row (none: no pick);
 *     rows i and j that picked each other become a pair.  The rounds stop
 *     after one that forms no pair.
 *  3. A row left unmatched joins the pair of its strongest coupling to a
 *     matched row, if it has one; otherwise it stays alone.  The leader of
 *     a pair is its smaller row; an aggregate is a pair with the rows that
 *     joined it, or a lone row.  Aggregates are numbered by their leaders,
 *     ascending: agg[i] is row i's coarse row.  No aggregate formed (every
 *     row alone) is an error.
 *  4. Galerkin coarse matrix A_c = P^T A P with P[i][agg[i]] = 1: the entry
 *     (I, J) exists when some entry (i, j) of A has agg[i] = I, agg[j] = J;
 *     its value sums those entries' values from 0 in ascending CSR position.
 *     Columns ascending.  dinv = 1 / diagonal on every level.
 *  5. The coarsest matrix (n <= coarse_max) is inverted densely by
 *     Gauss-Jordan without pivoting in the textbook order (as the block
 *     inverses above; A is SPD so every pivot is positive).
 *
 * Application y = V_l(r) on level l:
 *  - coarsest: y_i = sum over j ascending of Cinv[i][j] r_j, from 0;
 *  - l even ("smoothed"): x_i = omega (dinv_i r_i);
 *    t_i = r_i - (A x)_i;  r'_I = sum of t_i over the members i of
 *    aggregate I, ascending, from 0;  x_i = x_i + V_{l+1}(r')_{agg[i]};
 *    y_i = x_i + omega (dinv_i (r_i - (A x)_i));
 *  - l odd: r'_I = sum of r_i over the members, ascending, from 0;
 *    y_i = V_{l+1}(r')_{agg[i]}.
 * (A x)_i is the row sum of the products in column order, from 0, as in
 * or_spmv.  The operator r -> V_0(r) is linear and symmetric (the sweeps
 * before and after the correction are each other's adjoints, and the coarse
 * correction is P A_c^-1 P^T on the next level); it is the PCG
 * preconditioner M^-1.  Refresh: new level-0 values on the same pattern
 * keep the aggregates and patterns and recompute every coarse value, dinv
 * and the coarsest inverse (steps 4-5).
 * ------------------------------------------------------------------------ */
#define OR_ERR_UNSUPPORTED (-5)
#define OR_AMG_MAX_LEVELS 40
#define OR_AMG_ROUNDS 16

typedef struct {
    int64_t n, nnz;
    int32_t *row_ptr, *col;
    double *val, *dinv;
    int32_t *agg;       /* [n] coarse row of each row (all but the coarsest) */
    int32_t *mem_ptr;   /* [n_c + 1] members of each coarse row, ascending */
    int32_t *mem;       /* [n] */
    int32_t *cptr;      /* [nnz_c + 1] the coarse entry e sums val[cpos[cptr[e] .. cptr[e+1])] */
    int32_t *cpos;      /* [nnz] */
} or_level;

typedef struct {
    int n_levels;
    double omega;
    or_level lev[OR_AMG_MAX_LEVELS];
    double* cinv;       /* dense inverse of the coarsest matrix, row-major */
} or_amg;

static uint32_t or_fmix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return x;
}

typedef struct {
    double w;
    uint32_t h;
    int64_t lo, hi;
} or_key;

static or_key or_coupling(int64_t i, int64_t j, double a)
{
    or_key k;
    k.w = -a;
    k.lo = i < j ? i : j;
    k.hi = i < j ? j : i;
    k.h = or_fmix32((uint32_t)k.lo * 0x9E3779B1u + (uint32_t)k.hi);
    return k;
}

static int or_stronger(const or_key* a, const or_key* b)
{
    if (a->w != b->w) return a->w > b->w;
    if (a->h != b->h) return a->h > b->h;
    if (a->lo != b->lo) return a->lo < b->lo;
    return a->hi < b->hi;
}

/* strongest coupling of row i to a row j with (mate[j] >= 0) == want_matched; -1 if none */
static int64_t or_strongest(const or_level* L, int64_t i, const int32_t* mate, int want_matched)
{
    int64_t best = -1;
    or_key kb = {0.0, 0u, 0, 0};
    for (int64_t p = L->row_ptr[i]; p < L->row_ptr[i + 1]; ++p) {
        const int64_t j = L->col[p];
        if (j == i || !(L->val[p] < 0.0)) continue;
        if ((mate[j] >= 0) != want_matched) continue;
        const or_key k = or_coupling(i, j, L->val[p]);
        if (best < 0 || or_stronger(&k, &kb)) {
            best = j;
            kb = k;
        }
    }
    return best;
}

static void or_level_free(or_level* L)
{
    free(L->row_ptr); free(L->col); free(L->val); free(L->dinv);
    free(L->agg); free(L->mem_ptr); free(L->mem); free(L->cptr); free(L->cpos);
    memset(L, 0, sizeof(*L));
}

/* steps 1-3: agg[] of level L; returns the number of aggregates */
static int64_t or_aggregate(const or_level* L, int32_t* agg)
{
    const int64_t n = L->n;
    int32_t* mate = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t* pick = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t* leader = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i) mate[i] = -1;
    for (int round = 0; round < OR_AMG_ROUNDS; ++round) {
        for (int64_t i = 0; i < n; ++i) pick[i] = mate[i] >= 0 ? -1 : (int32_t)or_strongest(L, i, mate, 0);
        int64_t pairs = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int32_t j = pick[i];
            if (j >= 0 && pick[j] == (int32_t)i) {
                mate[i] = j;
                ++pairs;
            }
        }
        if (pairs == 0) break;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (mate[i] >= 0) {
            leader[i] = (int32_t)(i < mate[i] ? i : mate[i]);
        } else {
            const int64_t j = or_strongest(L, i, mate, 1);
            leader[i] = j >= 0 ? (j < mate[j] ? (int32_t)j : mate[j]) : (int32_t)i;
        }
    }
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i)
        if (leader[i] == (int32_t)i) pick[i] = (int32_t)nc++;   /* pick[] reused: id of a leader */
    for (int64_t i = 0; i < n; ++i) agg[i] = pick[leader[i]];
    free(mate); free(pick); free(leader);
    return nc;
}

/* step 4, pattern: C's row_ptr/col, L's members and contributions */
static void or_galerkin_pattern(or_level* L, or_level* C)
{
    const int64_t n = L->n, nc = C->n;
    L->mem_ptr = (int32_t*)calloc((size_t)(nc + 1), sizeof(int32_t));
    L->mem = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i) L->mem_ptr[L->agg[i] + 1]++;
    for (int64_t I = 0; I < nc; ++I) L->mem_ptr[I + 1] += L->mem_ptr[I];
    int32_t* fill = (int32_t*)calloc((size_t)(nc + 1), sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) L->mem[L->mem_ptr[L->agg[i]] + fill[L->agg[i]]++] = (int32_t)i;
    free(fill);
    /* per coarse row: the (J, position) pairs of its members' entries, sorted */
    int64_t* key = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L->nnz + 1));
    C->row_ptr = (int32_t*)calloc((size_t)(nc + 1), sizeof(int32_t));
    C->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(L->nnz + 1));
    L->cpos = (int32_t*)malloc(sizeof(int32_t) * (size_t)(L->nnz + 1));
    L->cptr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(L->nnz + 2));
    int64_t nk = 0, ne = 0;
    for (int64_t I = 0; I < nc; ++I) {
        const int64_t k0 = nk;
        for (int64_t m = L->mem_ptr[I]; m < L->mem_ptr[I + 1]; ++m) {
            const int64_t i = L->mem[m];
            for (int64_t p = L->row_ptr[i]; p < L->row_ptr[i + 1]; ++p)
                key[nk++] = ((int64_t)L->agg[L->col[p]] << 32) | p;
        }
        for (int64_t a = k0 + 1; a < nk; ++a) {   /* insertion sort of the row's keys */
            const int64_t v = key[a];
            int64_t b = a;
            while (b > k0 && key[b - 1] > v) { key[b] = key[b - 1]; --b; }
            key[b] = v;
        }
        for (int64_t a = k0; a < nk; ++a) {
            const int32_t J = (int32_t)(key[a] >> 32);
            if (a == k0 || J != (int32_t)(key[a - 1] >> 32)) {
                L->cptr[ne] = (int32_t)a;
                C->col[ne++] = J;
            }
            L->cpos[a] = (int32_t)(key[a] & 0xFFFFFFFF);
        }
        C->row_ptr[I + 1] = (int32_t)ne;
    }
    L->cptr[ne] = (int32_t)nk;
    C->nnz = ne;
    free(key);
}

/* step 4, values; dinv of C */
static int or_galerkin_values(const or_level* L, or_level* C)
{
    for (int64_t e = 0; e < C->nnz; ++e) {
        double s = 0.0;
        for (int64_t t = L->cptr[e]; t < L->cptr[e + 1]; ++t) s += L->val[L->cpos[t]];
        C->val[e] = s;
    }
    for (int64_t I = 0; I < C->n; ++I) {
        double d = 0.0;
        for (int64_t p = C->row_ptr[I]; p < C->row_ptr[I + 1]; ++p)
            if (C->col[p] == I) d = C->val[p];
        if (!(d > 0.0) || !isfinite(d)) return OR_ERR_BREAKDOWN;
        C->dinv[I] = 1.0 / d;
    }
    return OR_OK;
}

/* step 5 */
static int or_dense_inverse(const or_level* L, double* out)
{
    const int64_t n = L->n;
    double* W = (double*)calloc((size_t)(n * n + 1), sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) out[i * n + j] = (i == j) ? 1.0 : 0.0;
        for (int64_t p = L->row_ptr[i]; p < L->row_ptr[i + 1]; ++p) W[i * n + L->col[p]] = L->val[p];
    }
    int status = OR_OK;
    for (int64_t k = 0; k < n && status == OR_OK; ++k) {
        const double piv = W[k * n + k];
        if (!(piv > 0.0) || !isfinite(piv)) { status = OR_ERR_BREAKDOWN; break; }
        for (int64_t j = 0; j < n; ++j) {
            W[k * n + j] = W[k * n + j] / piv;
            out[k * n + j] = out[k * n + j] / piv;
        }
        for (int64_t i = 0; i < n; ++i) {
            if (i == k) continue;
            const double f = W[i * n + k];
            for (int64_t j = 0; j < n; ++j) {
                W[i * n + j] = W[i * n + j] - f * W[k * n + j];
                out[i * n + j] = out[i * n + j] - f * out[k * n + j];
            }
        }
    }
    free(W);
    return status;
}

static int or_amg_values(or_amg* h)
{
    for (int l = 0; l + 1 < h->n_levels; ++l) {
        const int st = or_galerkin_values(&h->lev[l], &h->lev[l + 1]);
        if (st != OR_OK) return st;
    }
    return or_dense_inverse(&h->lev[h->n_levels - 1], h->cinv);
}

void or_amg_free(void* handle)
{
    or_amg* h = (or_amg*)handle;
    if (!h) return;
    for (int l = 0; l < h->n_levels; ++l) or_level_free(&h->lev[l]);
    free(h->cinv);
    free(h);
}

/* the hierarchy of the CSR matrix (n, row_ptr, col, val); NULL with *status
 * set on failure (OR_ERR_UNSUPPORTED: coarsening stalled or too many levels;
 * OR_ERR_BREAKDOWN: a coarse diagonal or pivot not positive) */
void* or_amg_build(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val, double omega,
                   int64_t coarse_max, int* status)
{
    or_amg* h = (or_amg*)calloc(1, sizeof(or_amg));
    h->omega = omega;
    or_level* L = &h->lev[0];
    L->n = n;
    L->nnz = row_ptr[n];
    L->row_ptr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    L->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(L->nnz + 1));
    L->val = (double*)malloc(sizeof(double) * (size_t)(L->nnz + 1));
    L->dinv = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    memcpy(L->row_ptr, row_ptr, sizeof(int32_t) * (size_t)(n + 1));
    memcpy(L->col, col, sizeof(int32_t) * (size_t)L->nnz);
    memcpy(L->val, val, sizeof(double) * (size_t)L->nnz);
    h->n_levels = 1;
    *status = OR_OK;
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            if (col[p] == i) d = val[p];
        if (!(d > 0.0) || !isfinite(d)) { *status = OR_ERR_BREAKDOWN; or_amg_free(h); return NULL; }
        L->dinv[i] = 1.0 / d;
    }
    while (h->lev[h->n_levels - 1].n > coarse_max) {
        if (h->n_levels == OR_AMG_MAX_LEVELS) { *status = OR_ERR_UNSUPPORTED; or_amg_free(h); return NULL; }
        or_level* F = &h->lev[h->n_levels - 1];
        or_level* C = &h->lev[h->n_levels];
        F->agg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(F->n + 1));
        C->n = or_aggregate(F, F->agg);
        if (C->n == F->n) { *status = OR_ERR_UNSUPPORTED; or_amg_free(h); return NULL; }
        or_galerkin_pattern(F, C);
        C->val = (double*)malloc(sizeof(double) * (size_t)(C->nnz + 1));
        C->dinv = (double*)malloc(sizeof(double) * (size_t)(C->n + 1));
        h->n_levels++;
        const int st = or_galerkin_values(F, C);
        if (st != OR_OK) { *status = st; or_amg_free(h); return NULL; }
    }
    const int64_t nL = h->lev[h->n_levels - 1].n;
    h->cinv = (double*)malloc(sizeof(double) * (size_t)(nL * nL + 1));
    const int st = or_dense_inverse(&h->lev[h->n_levels - 1], h->cinv);
    if (st != OR_OK) { *status = st; or_amg_free(h); return NULL; }
    return h;
}

/* new level-0 values on the same pattern: steps 4-5 again */
int or_amg_refresh(void* handle, const double* val)
{
    or_amg* h = (or_amg*)handle;
    or_level* L = &h->lev[0];
    memcpy(L->val, val, sizeof(double) * (size_t)L->nnz);
    for (int64_t i = 0; i < L->n; ++i) {
        double d = 0.0;
        for (int64_t p = L->row_ptr[i]; p < L->row_ptr[i + 1]; ++p)
            if (L->col[p] == i) d = L->val[p];
        if (!(d > 0.0) || !isfinite(d)) return OR_ERR_BREAKDOWN;
        L->dinv[i] = 1.0 / d;
    }
    return or_amg_values(h);
}

int or_amg_levels(const void* handle) { return ((const or_amg*)handle)->n_levels; }

void or_amg_level_sizes(const void* handle, int l, int64_t* n, int64_t* nnz)
{
    const or_level* L = &((const or_amg*)handle)->lev[l];
    *n = L->n;
    *nnz = L->nnz;
}

/* copies of level l's arrays (agg and members: [n] and [n_{l+1} + 1] / [n],
 * not on the coarsest level); NULL pointers are skipped */
void or_amg_level_get(const void* handle, int l, int32_t* row_ptr, int32_t* col, double* val, double* dinv,
                      int32_t* agg, int32_t* mem_ptr, int32_t* mem)
{
    const or_amg* h = (const or_amg*)handle;
    const or_level* L = &h->lev[l];
    if (row_ptr) memcpy(row_ptr, L->row_ptr, sizeof(int32_t) * (size_t)(L->n + 1));
    if (col) memcpy(col, L->col, sizeof(int32_t) * (size_t)L->nnz);
    if (val) memcpy(val, L->val, sizeof(double) * (size_t)L->nnz);
    if (dinv) memcpy(dinv, L->dinv, sizeof(double) * (size_t)L->n);
    if (l + 1 < h->n_levels) {
        if (agg) memcpy(agg, L->agg, sizeof(int32_t) * (size_t)L->n);
        if (mem_ptr) memcpy(mem_ptr, L->mem_ptr, sizeof(int32_t) * (size_t)(h->lev[l + 1].n + 1));
        if (mem) memcpy(mem, L->mem, sizeof(int32_t) * (size_t)L->n);
    }
}

void or_amg_coarse_inverse(const void* handle, double* out)
{
    const or_amg* h = (const or_amg*)handle;
    const int64_t n = h->lev[h->n_levels - 1].n;
    memcpy(out, h->cinv, sizeof(double) * (size_t)(n * n));
}

static void or_amg_apply(const or_amg* h, int l, const double* r, double* y)
{
    const or_level* L = &h->lev[l];
    const int64_t n = L->n;
    if (l == h->n_levels - 1) {
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += h->cinv[i * n + j] * r[j];
            y[i] = s;
        }
        return;
    }
    const int64_t nc = h->lev[l + 1].n;
    double* rc = (double*)calloc((size_t)(nc + 1), sizeof(double));
    double* ec = (double*)calloc((size_t)(nc + 1), sizeof(double));
    if (l % 2 == 1) {
        for (int64_t I = 0; I < nc; ++I) {
            double s = 0.0;
            for (int64_t m = L->mem_ptr[I]; m < L->mem_ptr[I + 1]; ++m) s += r[L->mem[m]];
            rc[I] = s;
        }
        or_amg_apply(h, l + 1, rc, ec);
        for (int64_t i = 0; i < n; ++i) y[i] = ec[L->agg[i]];
    } else {
        double* x = (double*)calloc((size_t)(n + 1), sizeof(double));
        double* t = (double*)calloc((size_t)(n + 1), sizeof(double));
        for (int64_t i = 0; i < n; ++i) x[i] = h->omega * (L->dinv[i] * r[i]);
        or_spmv(n, L->row_ptr, L->col, L->val, x, t);
        for (int64_t i = 0; i < n; ++i) t[i] = r[i] - t[i];
        for (int64_t I = 0; I < nc; ++I) {
            double s = 0.0;
            for (int64_t m = L->mem_ptr[I]; m < L->mem_ptr[I + 1]; ++m) s += t[L->mem[m]];
            rc[I] = s;
        }
        or_amg_apply(h, l + 1, rc, ec);
        for (int64_t i = 0; i < n; ++i) x[i] = x[i] + ec[L->agg[i]];
        or_spmv(n, L->row_ptr, L->col, L->val, x, t);
        for (int64_t i = 0; i < n; ++i) y[i] = x[i] + h->omega * (L->dinv[i] * (r[i] - t[i]));
        free(x); free(t);
    }
    free(rc); free(ec);
}

void or_amg_vcycle(const void* handle, const double* r, double* y)
{
    or_amg_apply((const or_amg*)handle, 0, r, y);
}

/* PCG exactly as or_pcg, with z = M^-1 r by the hierarchy's V-cycle (level
 * 0 of the hierarchy is the system matrix) */
int or_pcg_amg(const void* handle, const double* b, double* x, double tol, int64_t max_iter, int max_restarts,
               int64_t* out, double* res)
{
    const or_amg* h = (const or_amg*)handle;
    const or_level* L = &h->lev[0];
    const int64_t n = L->n;
    double* r = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* z = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* p = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* q = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int status = OR_NOT_CONVERGED;
    int64_t it = 0;
    int restarts = 0;
    const double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        status = OR_OK;
        goto done;
    }
    for (;;) {
        or_spmv(n, L->row_ptr, L->col, L->val, x, q);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        if (sqrt(dot(n, r, r)) <= tol * bnorm) { status = OR_OK; break; }
        or_amg_vcycle(h, r, z);
        for (int64_t i = 0; i < n; ++i) p[i] = z[i];
        double rz = dot(n, r, z);
        int passed = 0;
        while (it < max_iter) {
            or_spmv(n, L->row_ptr, L->col, L->val, p, q);
            const double pq = dot(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { status = OR_ERR_BREAKDOWN; goto done; }
            const double a = rz / pq;
            for (int64_t i = 0; i < n; ++i) x[i] += a * p[i];
            for (int64_t i = 0; i < n; ++i) r[i] -= a * q[i];
            ++it;
            if (sqrt(dot(n, r, r)) <= tol * bnorm) { passed = 1; break; }
            or_amg_vcycle(h, r, z);
            const double rz_new = dot(n, r, z);
            const double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
        if (!passed) break;
        if (or_true_relres(n, L->row_ptr, L->col, L->val, b, x) <= tol) { status = OR_OK; break; }
        if (restarts >= max_restarts) break;
        ++restarts;
    }
done:
    out[0] = it;
    out[1] = restarts;
    res[0] = or_true_relres(n, L->row_ptr, L->col, L->val, b, x);
    free(r); free(z); free(p); free(q);
    return status;
}

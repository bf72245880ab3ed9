// Solve order (opt-in, rp_plan_set_solve_order): CG, the mixed solvers and
// BiCGStab run on a reverse Cuthill-McKee renumbering of the fused local
// block.
//
// The fused row order is the ranks' own cell order (Sec. 3).  Where that
// order has no locality (a scrambled numbering), the SpMV's x gathers touch
// one cache line per lane and the SpMV runs far below the bandwidth it gets
// on a naturally ordered mesh.  Renumbering the rows so that coupled rows
// are close (Cuthill and McKee 1969, reversed as George 1971 proposed)
// restores that locality.  Everything outside the solve stays in fused
// order: the pattern, P, the update, rp_spmv and the gradients.  The
// renumbered copy is a second CSR matrix Q A Q^T (row k of it is fused row
// perm[k], columns renumbered and sorted); its values follow the fused
// values through one gather, refreshed when a solve finds them older than
// the last update (A^T's values, for the transposed BiCGStab solve, the
// same way).  b and x are permuted into and out of the solve.
//
// The renumbered matrix is the same operator in another basis, so the
// iteration is the same method; only the summation order of each row's
// products (ascending column in the new numbering) differs, hence the
// rounding.
#include <algorithm>
#include <utility>
#include <vector>

#include "device_util.hpp"

namespace rp {

namespace {

// o64[k] = v64[sig[k]], o32[k] = v32[sig[k]] (values in solve order), and
// od[i] = d[perm[i]] (Jacobi inverses)
__global__ void __launch_bounds__(VEC_BLOCK)
order_values(int64_t nnz, int32_t n, const int32_t* __restrict__ sig, const int32_t* __restrict__ perm,
             const double* __restrict__ v64, const float* __restrict__ v32, const double* __restrict__ d64,
             const float* __restrict__ d32, double* __restrict__ o64, float* __restrict__ o32,
             double* __restrict__ od64, float* __restrict__ od32) {
    const int64_t i0 = (int64_t)blockIdx.x * VEC_BLOCK + threadIdx.x, di = (int64_t)gridDim.x * VEC_BLOCK;
    for (int64_t k = i0; k < nnz; k += di) {
        const int32_t s = sig[k];
        o64[k] = v64[s];
        o32[k] = v32[s];
    }
    for (int64_t i = i0; i < n; i += di) {
        const int32_t q = perm[i];
        od64[i] = d64[q];
        od32[i] = d32[q];
    }
}

// o[k] = v[sig[k]]
__global__ void __launch_bounds__(VEC_BLOCK)
order_gather(int64_t nnz, const int32_t* __restrict__ sig, const double* __restrict__ v, double* __restrict__ o) {
    for (int64_t k = (int64_t)blockIdx.x * VEC_BLOCK + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * VEC_BLOCK)
        o[k] = v[sig[k]];
}

// y[k] = x[perm[k]]: fused order -> solve order
__global__ void __launch_bounds__(VEC_BLOCK)
order_in(int32_t n, const int32_t* __restrict__ perm, const double* __restrict__ x, double* __restrict__ y) {
    for (int32_t k = blockIdx.x * VEC_BLOCK + threadIdx.x; k < n; k += gridDim.x * VEC_BLOCK) y[k] = x[perm[k]];
}

// x[perm[k]] = y[k]: solve order -> fused order
__global__ void __launch_bounds__(VEC_BLOCK)
order_out(int32_t n, const int32_t* __restrict__ perm, const double* __restrict__ y, double* __restrict__ x) {
    for (int32_t k = blockIdx.x * VEC_BLOCK + threadIdx.x; k < n; k += gridDim.x * VEC_BLOCK) x[perm[k]] = y[k];
}

}  // namespace

// Reverse Cuthill-McKee order of the graph of a structurally symmetric
// pattern (diagonal entries ignored).  Each connected component, taken in
// order of its lowest row, starts from a pseudo-peripheral row (George and
// Liu 1979: repeated breadth-first sweeps from a row of least degree in the
// last level, while the number of levels grows); the breadth-first order
// visits the neighbours of each row by ascending degree, ties by index.  The
// whole order is then reversed.  perm[k] = the row placed at position k.
std::vector<int32_t> rcm_order(int32_t n, const int32_t* row_ptr, const int32_t* col) {
    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<uint8_t> placed(n, 0);
    std::vector<int32_t> mark(n, -1), level(n, 0), comp, nb;
    comp.reserve(n);
    int32_t stamp = 0;
    auto deg = [&](int32_t i) { return row_ptr[i + 1] - row_ptr[i]; };
    // sorted: visit each row's new neighbours by ascending degree (the final
    // sweep); the pseudo-peripheral search needs only the levels
    auto bfs = [&](int32_t root, bool sorted) {
        ++stamp;
        comp.clear();
        comp.push_back(root);
        mark[root] = stamp;
        level[root] = 0;
        for (size_t h = 0; h < comp.size(); ++h) {
            const int32_t u = comp[h];
            nb.clear();
            for (int32_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
                const int32_t v = col[j];
                if (v != u && !placed[v] && mark[v] != stamp) {
                    mark[v] = stamp;
                    nb.push_back(v);
                }
            }
            if (sorted)
                std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
                    return deg(a) != deg(b) ? deg(a) < deg(b) : a < b;
                });
            for (int32_t v : nb) {
                level[v] = level[u] + 1;
                comp.push_back(v);
            }
        }
    };
    for (int32_t s0 = 0; s0 < n; ++s0) {
        if (placed[s0]) continue;
        int32_t root = s0, depth = -1;
        for (int sweep = 0; sweep < 8; ++sweep) {
            bfs(root, false);
            const int32_t d = level[comp.back()];
            if (d <= depth) break;
            depth = d;
            int32_t best = comp.back();
            for (size_t h = comp.size(); h-- > 0 && level[comp[h]] == d;) {
                const int32_t v = comp[h];
                if (deg(v) < deg(best) || (deg(v) == deg(best) && v < best)) best = v;
            }
            root = best;
        }
        bfs(root, true);
        for (int32_t v : comp) {
            placed[v] = 1;
            order.push_back(v);
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

int order_build(rp_plan* p) {
    const int32_t n = (int32_t)p->n_rows;
    const int64_t nnz = p->nnz;
    std::vector<int32_t> rp_h(n + 1), col_h(nnz);
    RP_HIP_TRY(hipMemcpy(rp_h.data(), p->d_row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (nnz > 0) RP_HIP_TRY(hipMemcpy(col_h.data(), p->d_col, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> perm = rcm_order(n, rp_h.data(), col_h.data());
    std::vector<int32_t> inv(n);
    for (int32_t k = 0; k < n; ++k) inv[perm[k]] = k;
    std::vector<int32_t> rrp(n + 1), rcol(nnz + SPMV_PAD, 0), sig(nnz);
    std::vector<std::pair<int32_t, int32_t>> row;
    rrp[0] = 0;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t o = perm[k];
        row.clear();
        for (int32_t j = rp_h[o]; j < rp_h[o + 1]; ++j) row.emplace_back(inv[col_h[j]], j);
        std::sort(row.begin(), row.end());
        const int32_t b = rrp[k];
        for (size_t t = 0; t < row.size(); ++t) {
            rcol[b + t] = row[t].first;
            sig[b + t] = row[t].second;
        }
        rrp[k + 1] = b + (int32_t)row.size();
    }
    auto dev = [](void** d, size_t bytes) -> int {
        RP_HIP_TRY(hipMalloc(d, bytes > 0 ? bytes : 1));
        RP_HIP_TRY(hipMemset(*d, 0, bytes > 0 ? bytes : 1));
        return RP_OK;
    };
    RP_TRY(dev((void**)&p->d_ro_perm, n * sizeof(int32_t)));
    RP_TRY(dev((void**)&p->d_ro_row_ptr, (n + 1) * sizeof(int32_t)));
    RP_TRY(dev((void**)&p->d_ro_col, (nnz + SPMV_PAD) * sizeof(int32_t)));
    RP_TRY(dev((void**)&p->d_ro_sig, nnz * sizeof(int32_t)));
    RP_TRY(dev((void**)&p->d_ro_val64, (nnz + SPMV_PAD) * sizeof(double)));
    RP_TRY(dev((void**)&p->d_ro_val32, (nnz + SPMV_PAD) * sizeof(float)));
    RP_TRY(dev((void**)&p->d_ro_dinv64, n * sizeof(double)));
    RP_TRY(dev((void**)&p->d_ro_dinv32, n * sizeof(float)));
    RP_TRY(dev((void**)&p->d_ro_b, n * sizeof(double)));
    RP_TRY(dev((void**)&p->d_ro_x, n * sizeof(double)));
    RP_HIP_TRY(hipMemcpy(p->d_ro_perm, perm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
    RP_HIP_TRY(hipMemcpy(p->d_ro_row_ptr, rrp.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    RP_HIP_TRY(hipMemcpy(p->d_ro_col, rcol.data(), (nnz + SPMV_PAD) * sizeof(int32_t), hipMemcpyHostToDevice));
    if (nnz > 0) RP_HIP_TRY(hipMemcpy(p->d_ro_sig, sig.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
    p->h_ro_perm = std::move(perm);
    p->ro_version = -1;
    return RP_OK;
}

int solve_in_order(rp_plan* p, const double* b, double* x, const rp_solve_opts& o, rp_solve_info& info,
                   hipStream_t s) {
    const int32_t n = (int32_t)p->n_rows;
    const int g = vec_grid(n);
    if (p->has_values && p->ro_version != p->values_version) {
        hipLaunchKernelGGL(order_values, dim3(vec_grid(std::max<int64_t>(p->nnz, n))), dim3(VEC_BLOCK), 0, s,
                           p->nnz, n, p->d_ro_sig, p->d_ro_perm, p->d_val64, p->d_val32, p->d_dinv64,
                           p->d_dinv32, p->d_ro_val64, p->d_ro_val32, p->d_ro_dinv64, p->d_ro_dinv32);
        RP_HIP_TRY(hipGetLastError());
        p->ro_version = p->values_version;
    }
    if (o.method == RP_BICGSTAB && o.transpose && p->has_values) {
        // A^T's values on the fused pattern, then in solve order
        RP_TRY(build_transpose(p, s));
        if (!p->d_ro_valT) {
            RP_HIP_TRY(hipMalloc(&p->d_ro_valT, (p->nnz + SPMV_PAD) * sizeof(double)));
            RP_HIP_TRY(hipMemsetAsync(p->d_ro_valT, 0, (p->nnz + SPMV_PAD) * sizeof(double), s));
        }
        if (p->ro_valT_version != p->values_version) {
            hipLaunchKernelGGL(order_gather, dim3(vec_grid(p->nnz)), dim3(VEC_BLOCK), 0, s, p->nnz, p->d_ro_sig,
                               p->d_valT, p->d_ro_valT);
            RP_HIP_TRY(hipGetLastError());
            p->ro_valT_version = p->values_version;
        }
    }
    hipLaunchKernelGGL(order_in, dim3(g), dim3(VEC_BLOCK), 0, s, n, p->d_ro_perm, b, p->d_ro_b);
    if (!o.x0_zero) hipLaunchKernelGGL(order_in, dim3(g), dim3(VEC_BLOCK), 0, s, n, p->d_ro_perm, x, p->d_ro_x);
    RP_HIP_TRY(hipGetLastError());
    const int rc = o.method == RP_BICGSTAB ? solve_bicgstab(p, p->d_ro_b, p->d_ro_x, o, info, s, true)
                   : o.precision == RP_FP64
                       ? solve_fp64(p, p->d_ro_b, p->d_ro_x, o, info, s, true)
                       : solve_mixed(p, p->d_ro_b, p->d_ro_x, o, info, s, o.precision == RP_MIXED_RR, true);
    // the solvers leave an iterate in x on these outcomes; on the others they
    // stopped before touching it
    if (rc == RP_OK || rc == RP_NOT_CONVERGED || rc == RP_ERR_BREAKDOWN) {
        hipLaunchKernelGGL(order_out, dim3(g), dim3(VEC_BLOCK), 0, s, n, p->d_ro_perm, p->d_ro_x, x);
        RP_HIP_TRY(hipGetLastError());
    }
    return rc;
}

}  // namespace rp

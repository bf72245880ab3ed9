// Block-Jacobi preconditioner (the stronger preconditioner of the outlook in
// Sec. 5), with every block inside one CPU rank: each share rank's fused rows
// are cut into runs of bs consecutive rows (a rank's last run may be
// shorter), and M = blockdiag(A_bb).  Each diagonal block is inverted once
// per update by Gauss-Jordan elimination without pivoting (A is SPD, so are
// its diagonal blocks), in the textbook order on [W | Z], W = A_bb, Z = I:
// for each pivot k, row k of W and Z is divided by W[k][k], then every other
// row i, ascending, subtracts W[i][k] times row k.  The upper triangle of Z
// is kept and used for both triangles, so M^-1 is exactly symmetric:
//   minv[b * P + i * bs - i * (i - 1) / 2 + (j - i)], P = bs (bs + 1) / 2,
// 0 <= i <= j < m (unused entries 0), FP64 and an RNE FP32 copy.
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_util.hpp"

namespace rp {

namespace {

__global__ void clear_word(uint32_t* w) {
    if (threadIdx.x == 0) *w = 0u;
}

// one thread per block
__global__ void __launch_bounds__(64)
bj_inverse_kernel(int64_t nb, int32_t bs, const int32_t* __restrict__ start, const int32_t* __restrict__ row_ptr,
                  const int32_t* __restrict__ col, const double* __restrict__ val, double* __restrict__ minv64,
                  float* __restrict__ minv32, uint32_t* bad_flag) {
#pragma clang fp contract(off)
    const int64_t P = (int64_t)bs * (bs + 1) / 2;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s0 = start[b];
        const int32_t m = start[b + 1] - s0;
        double W[BJ_MAX][BJ_MAX], Z[BJ_MAX][BJ_MAX];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                W[i][j] = 0.0;
                Z[i][j] = i == j ? 1.0 : 0.0;
            }
        for (int i = 0; i < m; ++i)
            for (int32_t e = row_ptr[s0 + i]; e < row_ptr[s0 + i + 1]; ++e) {
                const int32_t c = col[e];
                if (c >= s0 && c < s0 + m) W[i][c - s0] = val[e];
            }
        bool ok = true;
        for (int k = 0; k < m && ok; ++k) {
            const double piv = W[k][k];
            if (!(piv > 0.0) || !isfinite(piv)) {
                ok = false;
                break;
            }
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
        if (!ok) atomicOr(bad_flag, 1u);
        double* o64 = minv64 + b * P;
        float* o32 = minv32 + b * P;
        for (int q = 0; q < P; ++q) {
            o64[q] = 0.0;
            o32[q] = 0.0f;
        }
        if (!ok) continue;
        for (int i = 0; i < m; ++i)
            for (int j = i; j < m; ++j) {
                const int q = i * bs - i * (i - 1) / 2 + (j - i);
                o64[q] = Z[i][j];
                o32[q] = (float)Z[i][j];
            }
    }
}

}  // namespace

// block starts: each share rank's rows in runs of bs
std::vector<int32_t> bj_starts(const rp_plan* p, int32_t bs) {
    std::vector<int32_t> st;
    for (int32_t s = 0; s < p->alpha; ++s)
        for (int32_t c = 0; c < p->n_cells[s]; c += bs) st.push_back(p->row0[s] + c);
    st.push_back((int32_t)p->n_rows);
    return st;
}

int alloc_z(rp_plan* p) {
    if (!p->d_z) RP_HIP_TRY(hipMalloc(&p->d_z, sizeof(double) * (size_t)std::max<int64_t>(p->n_rows, 1)));
    if (!p->d_z32) RP_HIP_TRY(hipMalloc(&p->d_z32, sizeof(float) * (size_t)std::max<int64_t>(p->n_rows, 1)));
    return RP_OK;
}

int bj_prepare(rp_plan* p, int32_t bs, hipStream_t s) {
    if (bs < 1 || bs > BJ_MAX) {
        set_error("block size %d outside 1..%d", bs, BJ_MAX);
        return RP_ERR_ARG;
    }
    if (p->bj_bs != bs) {
        const std::vector<int32_t> st = bj_starts(p, bs);
        const int64_t nb = (int64_t)st.size() - 1;
        const int64_t P = (int64_t)bs * (bs + 1) / 2;
        for (void* q : {(void*)p->d_bj_start, (void*)p->d_bj_minv64, (void*)p->d_bj_minv32})
            if (q) RP_HIP_TRY(hipFree(q));
        p->d_bj_start = nullptr;
        p->d_bj_minv64 = nullptr;
        p->d_bj_minv32 = nullptr;
        p->bj_bs = 0;
        RP_HIP_TRY(hipMalloc(&p->d_bj_start, sizeof(int32_t) * st.size()));
        RP_HIP_TRY(hipMalloc(&p->d_bj_minv64, sizeof(double) * std::max<int64_t>(nb * P, 1)));
        RP_HIP_TRY(hipMalloc(&p->d_bj_minv32, sizeof(float) * std::max<int64_t>(nb * P, 1)));
        RP_HIP_TRY(hipMemcpyAsync(p->d_bj_start, st.data(), sizeof(int32_t) * st.size(), hipMemcpyHostToDevice, s));
        RP_HIP_TRY(hipStreamSynchronize(s));
        p->bj_blocks = nb;
        p->bj_bs = bs;
        p->bj_version = -1;
        bool aligned = 64 % bs == 0 && (bs & (bs - 1)) == 0;
        for (int32_t c : p->n_cells) aligned = aligned && c % bs == 0;
        p->bj_aligned = aligned;
    }
    RP_TRY(alloc_z(p));
    if (!p->d_bj_flag) RP_HIP_TRY(hipMalloc(&p->d_bj_flag, sizeof(uint32_t)));
    if (p->bj_version == p->values_version) return RP_OK;
    hipLaunchKernelGGL(clear_word, dim3(1), dim3(64), 0, s, p->d_bj_flag);
    const int64_t nb = p->bj_blocks;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nb + 63) / 64, 16384));
    hipLaunchKernelGGL(bj_inverse_kernel, dim3(grid), dim3(64), 0, s, nb, bs, p->d_bj_start, p->d_row_ptr,
                       p->d_col, p->d_val64, p->d_bj_minv64, p->d_bj_minv32, p->d_bj_flag);
    RP_HIP_TRY(hipGetLastError());
    uint32_t bad = 0;
    RP_HIP_TRY(hipMemcpyAsync(&bad, p->d_bj_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    if (bad) {
        set_error("block-Jacobi: a diagonal block of size <= %d is not positive definite", bs);
        return RP_ERR_BREAKDOWN;
    }
    p->bj_version = p->values_version;
    return RP_OK;
}

}  // namespace rp

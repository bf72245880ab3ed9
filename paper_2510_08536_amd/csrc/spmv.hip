// Plain y = A x on the fused local block (FP64 or FP32 copy of the matrix).
#include "spmv.hpp"

namespace rp {

template <typename T>
__global__ void __launch_bounds__(SPMV_BLOCK)
spmv_kernel(int32_t n_rows, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
            const T* __restrict__ val, const T* __restrict__ x, T* __restrict__ y) {
    __shared__ T lds[SPMV_CAP];
    const GroupRange gr = block_groups(n_rows);
    for (int32_t g = gr.g0; g < gr.n_groups; g += gr.step) {
        const int32_t r0 = g * SPMV_BLOCK;
        const int32_t nr = min(SPMV_BLOCK, n_rows - r0);
        const T s = spmv_group_row(row_ptr, col, val, x, r0, nr, lds);
        if ((int32_t)threadIdx.x < nr) y[r0 + threadIdx.x] = s;
    }
}

int launch_spmv64(rp_plan* p, const double* x, double* y, hipStream_t s) {
    if (p->n_rows == 0) return RP_OK;
    hipLaunchKernelGGL(spmv_kernel<double>, dim3(spmv_grid(p->n_rows)), dim3(SPMV_BLOCK), 0, s,
                       (int32_t)p->n_rows, p->d_row_ptr, p->d_col, p->d_val64, x, y);
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

int launch_spmv32(rp_plan* p, const float* x, float* y, hipStream_t s) {
    if (p->n_rows == 0) return RP_OK;
    hipLaunchKernelGGL(spmv_kernel<float>, dim3(spmv_grid(p->n_rows)), dim3(SPMV_BLOCK), 0, s,
                       (int32_t)p->n_rows, p->d_row_ptr, p->d_col, p->d_val32, x, y);
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

}  // namespace rp

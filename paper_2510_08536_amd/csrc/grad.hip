// Adjoint value gradient: for A x = b and lambda = A^-T dL/dx, the gradient
// of L with respect to the coefficient in slot k, at matrix position
// (row, col), is -lambda[row] * x[col].  Computed row by row over the fused
// CSR and written back in slot order through P^-1, so the caller receives it
// in the same LDU order it supplied the values in.
#include "device_util.hpp"

namespace rp {

namespace {

__global__ void __launch_bounds__(VEC_BLOCK)
value_grad_kernel(int32_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                  const int32_t* __restrict__ perm_inv, const double* __restrict__ lambda,
                  const double* __restrict__ x, double* __restrict__ g) {
    for (int32_t i = blockIdx.x * VEC_BLOCK + threadIdx.x; i < n; i += gridDim.x * VEC_BLOCK) {
        const double li = lambda[i];
        for (int32_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) g[perm_inv[j]] = -li * x[col[j]];
    }
}

}  // namespace

int launch_value_grad(rp_plan* p, const double* lambda, const double* x, double* g, hipStream_t s) {
    if (p->n_rows == 0) return RP_OK;
    int64_t blocks = (p->n_rows + VEC_BLOCK - 1) / VEC_BLOCK;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(value_grad_kernel, dim3((int)blocks), dim3(VEC_BLOCK), 0, s, (int32_t)p->n_rows,
                       p->d_row_ptr, p->d_col, p->d_perm_inv, lambda, x, g);
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

}  // namespace rp

// Plain y = A x on the fused local block (FP64 or FP32 copy of the matrix).
#include "spmv.hpp"

namespace rp {

template <typename T, int NW>
__global__ void __launch_bounds__(SPMV_BLOCK)
spmv_kernel(int32_t n_rows, SpmvIdx ix, const T* __restrict__ val, const T* __restrict__ x, T* __restrict__ y,
            XWin w) {
    __shared__ __align__(16) T lds[SPMV_CAP];
    __shared__ T xs[XWinSize<NW>::value];
    GroupRange gr = block_groups(ix, n_rows);
    for (int32_t g = gr.g0; g < gr.n_groups; g += gr.step) {
        const int32_t r0 = g * SPMV_BLOCK;
        const int32_t nr = min(SPMV_BLOCK, n_rows - r0);
        const GroupRow<T> gr_ = spmv_group_row<T, NW>(ix, val, x, n_rows, g, nr, w, xs, lds, gr);
        if ((int32_t)threadIdx.x < nr) y[r0 + threadIdx.x] = gr_.s;
    }
}

template <typename T>
int launch_spmv(rp_plan* p, const T* val, const T* x, T* y, hipStream_t s) {
    if (p->n_rows == 0) return RP_OK;
    const XWin w{{p->xw_d[0], p->xw_d[1]}};
#define RP_LAUNCH(NW)                                                                                    \
    hipLaunchKernelGGL((spmv_kernel<T, NW>), dim3(spmv_grid(p->n_rows)), dim3(SPMV_BLOCK), 0, s,        \
                       (int32_t)p->n_rows, spmv_idx(p), val, x, y, w)
    RP_DISPATCH_NW(p->xw_mode, RP_LAUNCH);
#undef RP_LAUNCH
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

int launch_spmv64(rp_plan* p, const double* x, double* y, hipStream_t s) {
    return launch_spmv<double>(p, p->d_val64, x, y, s);
}

int launch_spmv32(rp_plan* p, const float* x, float* y, hipStream_t s) {
    return launch_spmv<float>(p, p->d_val32, x, y, s);
}

}  // namespace rp

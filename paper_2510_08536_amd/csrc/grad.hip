// Adjoint value gradient: for A x = b and lambda = A^-T dL/dx, the gradient
// of L with respect to the coefficient in slot k, at matrix position
// (row, col), is -lambda[row] * x[col].  Computed in slot order, so the
// caller receives it in the LDU order it supplied the values in and every
// read of the addressing and write of g is coalesced.  A rank's slots are its
// cells (position (c, c)), its upper faces (owner, neighbour), its lower
// faces (neighbour, owner) and its interface faces; rank s's cell c is row
// row0[s] + c.  An interface slot's column is read from the CSR pattern and
// its row is the column of its transposed partner (the partner rank's
// matching interface slot).
#include "device_util.hpp"

namespace rp {

namespace {

__device__ __forceinline__ int32_t find_rank(const int32_t* tab, int32_t n, int32_t v) {
    int32_t a = 0, b = n;
    while (b - a > 1) {
        const int32_t m = (a + b) >> 1;
        if (tab[m] <= v) a = m; else b = m;
    }
    return a;
}

__global__ void __launch_bounds__(VEC_BLOCK)
value_grad_kernel(int32_t n_slots, int32_t alpha, const int32_t* __restrict__ slot_off,
                  const int32_t* __restrict__ row0, const int32_t* __restrict__ nf,
                  const int32_t* __restrict__ face_off, const int32_t* __restrict__ owner,
                  const int32_t* __restrict__ nbr, const int32_t* __restrict__ iface_off,
                  const int32_t* __restrict__ partner, const int32_t* __restrict__ perm,
                  const int32_t* __restrict__ col, const double* __restrict__ lambda,
                  const double* __restrict__ x, double* __restrict__ g) {
    // contiguous chunk of slots per block: a thread's successive slots (256
    // apart) stay in one rank, whose tables it keeps in registers
    const int64_t per = (((int64_t)n_slots + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
    const int64_t a64 = (int64_t)blockIdx.x * per;
    const int32_t k0 = (int32_t)(a64 < n_slots ? a64 : n_slots);
    const int32_t k1 = (int32_t)(a64 + per < n_slots ? a64 + per : n_slots);
    int32_t lo = 0, hi = 0, nc = 0, f = 0, r0 = 0, fo = 0, io = 0;
    for (int32_t k = k0 + threadIdx.x; k < k1; k += VEC_BLOCK) {
        if (k < lo || k >= hi) {
            const int32_t s = find_rank(slot_off, alpha, k);
            lo = slot_off[s];
            hi = slot_off[s + 1];
            r0 = row0[s];
            nc = row0[s + 1] - r0;
            f = nf[s];
            fo = face_off[s];
            io = iface_off[s];
        }
        const int32_t loc = k - lo;
        int32_t r, c;
        if (loc < nc) {
            r = c = r0 + loc;
        } else if (loc < nc + f) {
            const int32_t e = fo + loc - nc;
            r = r0 + owner[e];
            c = r0 + nbr[e];
        } else if (loc < nc + 2 * f) {
            const int32_t e = fo + loc - nc - f;
            r = r0 + nbr[e];
            c = r0 + owner[e];
        } else {
            const int32_t kp = partner[io + (loc - nc - 2 * f)];
            if (kp < 0) {  // coupling outside the share: no local position
                g[k] = 0.0;
                continue;
            }
            c = col[perm[k]];
            r = col[perm[kp]];
        }
        g[k] = -lambda[r] * x[c];
    }
}

}  // namespace

int launch_value_grad(rp_plan* p, const double* lambda, const double* x, double* g, hipStream_t s) {
    if (p->n_slots == 0) return RP_OK;
    int64_t blocks = (p->n_slots + VEC_BLOCK * 64 - 1) / (VEC_BLOCK * 64);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(value_grad_kernel, dim3((int)blocks), dim3(VEC_BLOCK), 0, s, (int32_t)p->n_slots, p->alpha,
                       p->d_slot_off, p->d_row0, p->d_nf, p->d_face_off, p->d_owner, p->d_nbr, p->d_iface_off,
                       p->d_iface_partner, p->d_perm, p->d_col, lambda, x, g);
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

}  // namespace rp

// Coefficient update (Sec. 3, update procedure).
//
// The receive buffer holds the share's coefficients in slot order (ranks in
// order, each [diag | upper | lower | interface]).  The reorder by P is done
// in its gather form, val[pos] = buf[P^-1(pos)], so the matrix writes are
// coalesced and the reads follow the LDU regions each row draws from.  The
// same pass writes the FP32 copy (round to nearest even) and flags values
// that are not finite; a second grid part computes the Jacobi inverse
// diagonal as one IEEE division per row.
#include <algorithm>
#include <cmath>

#include "device_util.hpp"

namespace rp {

namespace {

__device__ __forceinline__ int32_t find_block(const int32_t* tab, int32_t n, int32_t v) {
    int32_t a = 0, b = n;
    while (b - a > 1) {
        const int32_t m = (a + b) >> 1;
        if (tab[m] <= v) a = m; else b = m;
    }
    return a;
}

constexpr int STAGE_RANKS = 60;  // rank pointers per staging launch (kernel-argument budget)

struct StageArgs {
    const double* src[STAGE_RANKS][4];   // diag, upper, lower (or upper), iface
    int32_t s0;                          // first share rank of this launch
    int32_t ns;                          // ranks in this launch
};

// copy ranks s0..s0+ns-1 from their own arrays into the receive buffer
__global__ void stage_kernel(StageArgs a, const int32_t* slot_off, const int32_t* row0, const int32_t* nf,
                             double* recv) {
    const int32_t k0 = slot_off[a.s0];
    const int32_t k1 = slot_off[a.s0 + a.ns];
    for (int32_t k = k0 + blockIdx.x * blockDim.x + threadIdx.x; k < k1; k += gridDim.x * blockDim.x) {
        const int32_t s = a.s0 + find_block(slot_off + a.s0, a.ns, k);
        const int32_t loc = k - slot_off[s];
        const int32_t nc = row0[s + 1] - row0[s];
        const int32_t f = nf[s];
        const int ls = s - a.s0;
        double v;
        if (loc < nc) v = a.src[ls][0][loc];
        else if (loc < nc + f) v = a.src[ls][1][loc - nc];
        else if (loc < nc + 2 * f) v = a.src[ls][2][loc - nc - f];
        else v = a.src[ls][3][loc - nc - 2 * f];
        recv[k] = v;
    }
}

__global__ void scatter_kernel(int32_t n_pos, int32_t n_rows, int32_t alpha, const int32_t* __restrict__ perm_inv,
                               const double* __restrict__ recv, const int32_t* __restrict__ slot_off,
                               const int32_t* __restrict__ row0, double* __restrict__ val64,
                               float* __restrict__ val32, double* __restrict__ dinv64,
                               float* __restrict__ dinv32, uint32_t* flags) {
    bool bad = false;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_pos; j += stride) {
        const double v = recv[perm_inv[j]];
        __builtin_nontemporal_store(v, val64 + j);
        __builtin_nontemporal_store((float)v, val32 + j);
        bad |= !isfinite(v);
    }
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_rows; i += stride) {
        const int32_t s = find_block(row0, alpha, i);
        const double d = recv[slot_off[s] + (i - row0[s])];
        const double inv = 1.0 / d;
        dinv64[i] = inv;
        dinv32[i] = (float)inv;
        bad |= !(d > 0.0) || !isfinite(d);
    }
    if (bad) atomicOr(flags, (uint32_t)FLAG_VALUE);
}

// flags[1] |= 1 when upper != lower for some face, or an interface value
// differs (bitwise) from its partner's
__global__ void symmetry_kernel(int32_t n_faces, int32_t n_iface, int32_t alpha, bool check_faces,
                                const double* __restrict__ recv, const int32_t* __restrict__ slot_off,
                                const int32_t* __restrict__ row0, const int32_t* __restrict__ nf,
                                const int32_t* __restrict__ face_off, const int32_t* __restrict__ iface_off,
                                const int32_t* __restrict__ partner, uint32_t* flags) {
    bool asym = false;
    const int32_t stride = gridDim.x * blockDim.x;
    if (check_faces) {
        for (int32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < n_faces; f += stride) {
            const int32_t s = find_block(face_off, alpha, f);
            const int32_t k = slot_off[s] + (row0[s + 1] - row0[s]) + (f - face_off[s]);
            asym |= __double_as_longlong(recv[k]) != __double_as_longlong(recv[k + nf[s]]);
        }
    }
    for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n_iface; e += stride) {
        const int32_t k2 = partner[e];
        if (k2 < 0) continue;
        const int32_t s = find_block(iface_off, alpha, e);
        const int32_t k = slot_off[s] + (row0[s + 1] - row0[s]) + 2 * nf[s] + (e - iface_off[s]);
        asym |= __double_as_longlong(recv[k]) != __double_as_longlong(recv[k2]);
    }
    if (asym) atomicOr(flags + 1, 1u);
}

int grid_for(int64_t n, int block = 256, int cap = 8192) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// Values of A^T on the fused pattern: entry (i, j) takes A(j, i), found by a
// binary search for column i in row j (columns ascend within a row).  An
// entry without a partner sets *missing.
__global__ void transpose_values(int32_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                 const double* __restrict__ val, double* __restrict__ valT,
                                 uint32_t* __restrict__ missing) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col[e];
            int32_t a = row_ptr[j], b = row_ptr[j + 1];
            while (a < b) {
                const int32_t m = (a + b) >> 1;
                if (col[m] < i) a = m + 1;
                else b = m;
            }
            if (a < row_ptr[j + 1] && col[a] == i) {
                valT[e] = val[a];
            } else {
                valT[e] = 0.0;
                atomicOr(missing, 1u);
            }
        }
    }
}

}  // namespace

// A^T's values into d_valT, unless they are current (same values_version)
int build_transpose(rp_plan* p, hipStream_t s) {
    if (p->d_valT != nullptr && p->valT_version == p->values_version) return RP_OK;
    if (p->d_valT == nullptr) {
        RP_HIP_TRY(hipMalloc(&p->d_valT, sizeof(double) * ((size_t)p->nnz + SPMV_PAD)));
        RP_HIP_TRY(hipMemsetAsync(p->d_valT + p->nnz, 0, sizeof(double) * SPMV_PAD, s));
        RP_HIP_TRY(hipMalloc(&p->d_tflag, sizeof(uint32_t)));
    }
    RP_HIP_TRY(hipMemsetAsync(p->d_tflag, 0, sizeof(uint32_t), s));
    const int32_t n = (int32_t)p->n_rows;
    const int grid = (int)std::min<int64_t>((p->n_rows + 255) / 256, 4096);
    hipLaunchKernelGGL(transpose_values, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, n, p->d_row_ptr, p->d_col,
                       p->d_val64, p->d_valT, p->d_tflag);
    RP_HIP_TRY(hipGetLastError());
    uint32_t missing = 0;
    RP_HIP_TRY(hipMemcpyAsync(&missing, p->d_tflag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    if (missing) {
        set_error("the fused pattern is not structurally symmetric: A^T has entries outside it");
        return RP_ERR_UNSUPPORTED;
    }
    p->valT_version = p->values_version;
    return RP_OK;
}

int launch_stage_table(rp_plan* p, bool lower_given, hipStream_t s) {
    for (int32_t s0 = 0; s0 < p->alpha; s0 += STAGE_RANKS) {
        StageArgs a;
        a.s0 = s0;
        a.ns = std::min(STAGE_RANKS, p->alpha - s0);
        for (int i = 0; i < a.ns; ++i) {
            const int32_t r = s0 + i;
            a.src[i][0] = p->h_src[4 * r + 0];
            a.src[i][1] = p->h_src[4 * r + 1];
            a.src[i][2] = lower_given ? p->h_src[4 * r + 2] : p->h_src[4 * r + 1];
            a.src[i][3] = p->h_src[4 * r + 3];
        }
        const int64_t len = (int64_t)p->slot_off[s0 + a.ns] - p->slot_off[s0];
        if (len == 0) continue;
        hipLaunchKernelGGL(stage_kernel, dim3(grid_for(len)), dim3(256), 0, s, a, p->d_slot_off, p->d_row0,
                           p->d_nf, p->d_recv);
        RP_HIP_TRY(hipGetLastError());
    }
    return RP_OK;
}

int launch_update(rp_plan* p, const double* src, hipStream_t s) {
    const int64_t n_pos = p->n_slots;
    if (n_pos == 0 && p->n_rows == 0) return RP_OK;
    const int g = grid_for(std::max<int64_t>(n_pos, p->n_rows));
    RP_TRY(timing_begin(p, RP_KERNEL_SCATTER, s));
    hipLaunchKernelGGL(scatter_kernel, dim3(g), dim3(256), 0, s, (int32_t)n_pos, (int32_t)p->n_rows, p->alpha,
                       p->d_perm_inv, src, p->d_slot_off, p->d_row0, p->d_val64, p->d_val32,
                       p->d_dinv64, p->d_dinv32, p->d_flags);
    RP_HIP_TRY(hipGetLastError());
    RP_TRY(timing_end(p, RP_KERNEL_SCATTER, s));
    return RP_OK;
}

int launch_symmetry_check(rp_plan* p, const double* src, bool lower_given, hipStream_t s) {
    int64_t total_faces = 0;
    for (int32_t f : p->n_faces) total_faces += f;
    const int64_t work = std::max<int64_t>(lower_given ? total_faces : 0, p->n_iface_share);
    if (work == 0) return RP_OK;
    hipLaunchKernelGGL(symmetry_kernel, dim3(grid_for(work)), dim3(256), 0, s, (int32_t)total_faces,
                       (int32_t)p->n_iface_share, p->alpha, lower_given, src, p->d_slot_off, p->d_row0,
                       p->d_nf, p->d_face_off, p->d_iface_off, p->d_iface_partner, p->d_flags);
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

}  // namespace rp

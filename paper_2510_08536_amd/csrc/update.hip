// Coefficient update (Sec. 3, update procedure).
//
// The receive buffer holds the share's coefficients in slot order (ranks in
// order, each [diag | upper | lower | interface]).  The reorder by P is done
// in its gather form, val[pos] = buf[P^-1(pos)], so the matrix writes are
// coalesced and the reads follow the LDU regions each row draws from.  The
// same pass writes the FP32 copy (round to nearest even) and flags values
// that are not finite; a second grid part computes the Jacobi inverse
// diagonal as one IEEE division per row.
//
// Where the buffer is real (values that came from host memory, or a buffer
// the caller filled) the kernels read it; for per-rank arrays in device
// memory it stays virtual, and the same gather reads each slot straight
// from its rank's array through a table of 4 pointers per rank.
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

// ---------------------------------------------------------------------------
// Device-resident per-rank arrays: the receive buffer stays virtual.  Slot k
// of rank s at local offset loc lies in that rank's diag, upper, lower or
// interface array (table[4 s + region]); the gather reads it from there
// instead of from a staged copy.  Positions are taken in contiguous chunks
// per block, so one thread's successive positions (256 apart) almost always
// come from the same rank, whose slot range each thread keeps in registers.
// ---------------------------------------------------------------------------
struct RankSlots {
    int32_t s = -1, k_lo = 0, k_hi = 0, nc = 0, nf = 0;
};

__device__ __forceinline__ void rank_of_slot(RankSlots& r, int32_t k, int32_t alpha, const int32_t* slot_off,
                                             const int32_t* row0, const int32_t* nf) {
    if (k >= r.k_lo && k < r.k_hi) return;
    r.s = find_block(slot_off, alpha, k);
    r.k_lo = slot_off[r.s];
    r.k_hi = slot_off[r.s + 1];
    r.nc = row0[r.s + 1] - row0[r.s];
    r.nf = nf[r.s];
}

// the value of slot k (rank r.s) from the per-rank arrays
__device__ __forceinline__ double slot_value(const RankSlots& r, int32_t k, const double* const* table) {
    const int32_t loc = k - r.k_lo;
    int reg, base;
    if (loc < r.nc) { reg = 0; base = 0; }
    else if (loc < r.nc + r.nf) { reg = 1; base = r.nc; }
    else if (loc < r.nc + 2 * r.nf) { reg = 2; base = r.nc + r.nf; }
    else { reg = 3; base = r.nc + 2 * r.nf; }
    return table[4 * r.s + reg][loc - base];
}

__device__ __forceinline__ void block_chunk(int64_t n, int32_t& a, int32_t& b) {
    const int64_t per = ((n + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
    const int64_t a64 = (int64_t)blockIdx.x * per;
    a = (int32_t)(a64 < n ? a64 : n);
    b = (int32_t)(a64 + per < n ? a64 + per : n);
}

// val64[j] = value of slot P^-1(j), val32 = RNE, dinv = 1 / diag, straight
// from the per-rank arrays; same values and flags as scatter_kernel on the
// staged buffer
__global__ void __launch_bounds__(256)
gather_kernel(int32_t n_pos, int32_t n_rows, int32_t alpha, const int32_t* __restrict__ perm_inv,
              const double* const* __restrict__ table, const int32_t* __restrict__ slot_off,
              const int32_t* __restrict__ row0, const int32_t* __restrict__ nf, double* __restrict__ val64,
              float* __restrict__ val32, double* __restrict__ dinv64, float* __restrict__ dinv32,
              uint32_t* flags) {
    bool bad = false;
    int32_t j0, j1;
    block_chunk(n_pos, j0, j1);
    RankSlots rs;
    constexpr int U = 4;
    int32_t j = j0 + threadIdx.x;
    for (; j + (U - 1) * 256 < j1; j += U * 256) {
        int32_t k[U];
#pragma unroll
        for (int u = 0; u < U; ++u) k[u] = perm_inv[j + u * 256];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            rank_of_slot(rs, k[u], alpha, slot_off, row0, nf);
            v[u] = slot_value(rs, k[u], table);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            __builtin_nontemporal_store(v[u], val64 + j + u * 256);
            __builtin_nontemporal_store((float)v[u], val32 + j + u * 256);
            bad |= !isfinite(v[u]);
        }
    }
    for (; j < j1; j += 256) {
        const int32_t k = perm_inv[j];
        rank_of_slot(rs, k, alpha, slot_off, row0, nf);
        const double v = slot_value(rs, k, table);
        __builtin_nontemporal_store(v, val64 + j);
        __builtin_nontemporal_store((float)v, val32 + j);
        bad |= !isfinite(v);
    }
    int32_t i0, i1;
    block_chunk(n_rows, i0, i1);
    int32_t s = -1, lo = 0, hi = 0;
    for (int32_t i = i0 + threadIdx.x; i < i1; i += 256) {
        if (i < lo || i >= hi) {
            s = find_block(row0, alpha, i);
            lo = row0[s];
            hi = row0[s + 1];
        }
        const double d = table[4 * s][i - lo];
        const double inv = 1.0 / d;
        dinv64[i] = inv;
        dinv32[i] = (float)inv;
        bad |= !(d > 0.0) || !isfinite(d);
    }
    if (bad) atomicOr(flags, (uint32_t)FLAG_VALUE);
}

// symmetry_kernel on the per-rank arrays: flags[1] |= 1 when upper != lower
// (check_faces) or an interface value differs from its partner's
__global__ void __launch_bounds__(256)
symmetry_gather_kernel(int32_t n_faces, int32_t n_iface, int32_t alpha, bool check_faces,
                       const double* const* __restrict__ table, const int32_t* __restrict__ slot_off,
                       const int32_t* __restrict__ row0, const int32_t* __restrict__ nf,
                       const int32_t* __restrict__ face_off, const int32_t* __restrict__ iface_off,
                       const int32_t* __restrict__ partner, uint32_t* flags) {
    bool asym = false;
    if (check_faces) {
        int32_t f0, f1;
        block_chunk(n_faces, f0, f1);
        int32_t s = -1, lo = 0, hi = 0;
        for (int32_t f = f0 + threadIdx.x; f < f1; f += 256) {
            if (f < lo || f >= hi) {
                s = find_block(face_off, alpha, f);
                lo = face_off[s];
                hi = face_off[s + 1];
            }
            asym |= __double_as_longlong(table[4 * s + 1][f - lo]) != __double_as_longlong(table[4 * s + 2][f - lo]);
        }
    }
    int32_t e0, e1;
    block_chunk(n_iface, e0, e1);
    int32_t s = -1, lo = 0, hi = 0;
    RankSlots rp;
    for (int32_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const int32_t k2 = partner[e];
        if (k2 < 0) continue;
        if (e < lo || e >= hi) {
            s = find_block(iface_off, alpha, e);
            lo = iface_off[s];
            hi = iface_off[s + 1];
        }
        rank_of_slot(rp, k2, alpha, slot_off, row0, nf);
        asym |= __double_as_longlong(table[4 * s + 3][e - lo]) != __double_as_longlong(slot_value(rp, k2, table));
    }
    if (asym) atomicOr(flags + 1, 1u);
}

__global__ void clear_flags(uint32_t* flags) {
    if (threadIdx.x < 2) flags[threadIdx.x] = 0u;
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

int launch_clear_flags(uint32_t* flags, hipStream_t s) {
    hipLaunchKernelGGL(clear_flags, dim3(1), dim3(64), 0, s, flags);
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

int launch_update_gather(rp_plan* p, const double* const* table, bool lower_given, uint32_t* flags,
                         hipStream_t s) {
    int64_t total_faces = 0;
    for (int32_t f : p->n_faces) total_faces += f;
    const int64_t work = std::max<int64_t>(lower_given ? total_faces : 0, p->n_iface_share);
    if (work > 0) {
        hipLaunchKernelGGL(symmetry_gather_kernel, dim3(grid_for(work, 256, 2048)), dim3(256), 0, s,
                           (int32_t)total_faces, (int32_t)p->n_iface_share, p->alpha, lower_given, table,
                           p->d_slot_off, p->d_row0, p->d_nf, p->d_face_off, p->d_iface_off, p->d_iface_partner,
                           flags);
        RP_HIP_TRY(hipGetLastError());
    }
    const int64_t n_pos = p->n_slots;
    if (n_pos == 0 && p->n_rows == 0) return RP_OK;
    const int g = grid_for(std::max<int64_t>(n_pos, p->n_rows), 256, 2048);
    RP_TRY(timing_begin(p, RP_KERNEL_SCATTER, s));
    hipLaunchKernelGGL(gather_kernel, dim3(g), dim3(256), 0, s, (int32_t)n_pos, (int32_t)p->n_rows, p->alpha,
                       p->d_perm_inv, table, p->d_slot_off, p->d_row0, p->d_nf, p->d_val64, p->d_val32,
                       p->d_dinv64, p->d_dinv32, flags);
    RP_HIP_TRY(hipGetLastError());
    RP_TRY(timing_end(p, RP_KERNEL_SCATTER, s));
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

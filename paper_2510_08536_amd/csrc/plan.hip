// Repartitioning plan on the GPU (Sec. 3: steps 1-3 and the three resulting
// structures: fused pattern, update pattern U, permutation P).
//
// Every LDU coefficient of the share's ranks is one slot of the receive
// buffer, in the order [rank][diag | upper | lower | interface].  A slot's
// matrix position follows from the rank's addressing alone:
//   diag  c  -> (row0 + c,        lo + row0 + c)
//   upper f  -> (row0 + owner_f,  lo + row0 + nbr_f)
//   lower f  -> (row0 + nbr_f,    lo + row0 + owner_f)
//   iface e  -> (row0 + cell_e,   off_q + ncell_e)     q = nbr rank of e
// with lo = first fused global row and row0 = the rank's first fused row.  A
// slot is local when its global column lies in the fused row range (the
// localisation rule of Sec. 3), non-local otherwise.
//
// The build is a counting sort of slots by row, then a per-row sort by
// column; columns within a row are unique (a repeat is a mesh error), so the
// result, and with it P, does not depend on the order in which the atomics
// placed the slots.
#include <algorithm>
#include <unordered_map>

#include "spmv.hpp"

namespace rp {

namespace {

enum SlotKind : int32_t { K_INVALID = -1, K_DIAG = 0, K_UPPER = 1, K_LOWER = 2, K_IFACE = 3 };

struct ShareTables {
    const int32_t* slot_off;    // [alpha+1]
    const int32_t* row0;        // [alpha+1]
    const int32_t* nf;          // [alpha]
    const int32_t* face_off;    // [alpha+1]
    const int32_t* owner;       // [faces]
    const int32_t* nbr;         // [faces]
    const int32_t* iface_off;   // [alpha+1]
    const int32_t* if_cell;     // [ifaces]
    const int32_t* if_rank;
    const int32_t* if_ncell;
    const int64_t* off_all;     // [n_ranks_total+1]
    uint32_t* flags;
    int64_t lo, hi;
    int32_t alpha, first, n_ranks_total;
};

// largest s in [0, n) with tab[s] <= v   (tab ascending, tab[0] <= v)
__device__ __forceinline__ int32_t find_block(const int32_t* tab, int32_t n, int32_t v) {
    int32_t a = 0, b = n;  // invariant: tab[a] <= v, answer in [a, b)
    while (b - a > 1) {
        const int32_t m = (a + b) >> 1;
        if (tab[m] <= v) a = m; else b = m;
    }
    return a;
}

struct Slot {
    int32_t kind, s, row;
    int64_t colg;
};

__device__ Slot decode_slot(const ShareTables& t, int32_t k) {
    Slot o;
    o.s = find_block(t.slot_off, t.alpha, k);
    const int32_t loc = k - t.slot_off[o.s];
    const int32_t r0 = t.row0[o.s];
    const int32_t nc = t.row0[o.s + 1] - r0;
    const int32_t nf = t.nf[o.s];
    if (loc < nc) {
        o.kind = K_DIAG;
        o.row = r0 + loc;
        o.colg = t.lo + o.row;
        return o;
    }
    if (loc < nc + 2 * nf) {
        const bool up = loc < nc + nf;
        const int32_t f = t.face_off[o.s] + (up ? loc - nc : loc - nc - nf);
        const int32_t a = t.owner[f], b = t.nbr[f];
        if (a < 0 || a >= nc || b < 0 || b >= nc) {
            atomicOr(t.flags, (uint32_t)FLAG_MESH_RANGE);
            o.kind = K_INVALID;
            return o;
        }
        if (a == b) {
            atomicOr(t.flags, (uint32_t)FLAG_MESH_SELF);
            o.kind = K_INVALID;
            return o;
        }
        o.kind = up ? K_UPPER : K_LOWER;
        o.row = r0 + (up ? a : b);
        o.colg = t.lo + r0 + (up ? b : a);
        return o;
    }
    const int32_t e = t.iface_off[o.s] + (loc - nc - 2 * nf);
    const int32_t c = t.if_cell[e], q = t.if_rank[e], d = t.if_ncell[e];
    if (c < 0 || c >= nc || q < 0 || q >= t.n_ranks_total) {
        atomicOr(t.flags, (uint32_t)FLAG_MESH_RANGE);
        o.kind = K_INVALID;
        return o;
    }
    if (q == t.first + o.s) {
        atomicOr(t.flags, (uint32_t)FLAG_MESH_SELF);
        o.kind = K_INVALID;
        return o;
    }
    const int64_t qn = t.off_all[q + 1] - t.off_all[q];
    if (d < 0 || d >= qn) {
        atomicOr(t.flags, (uint32_t)FLAG_MESH_RANGE);
        o.kind = K_INVALID;
        return o;
    }
    o.kind = K_IFACE;
    o.row = r0 + c;
    o.colg = t.off_all[q] + d;
    return o;
}

__global__ void plan_count(ShareTables t, int32_t n_slots, int32_t* cnt, int32_t* nl_cnt) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_slots; k += gridDim.x * blockDim.x) {
        const Slot sl = decode_slot(t, k);
        if (sl.kind == K_INVALID) continue;
        if (sl.colg >= t.lo && sl.colg < t.hi) atomicAdd(cnt + sl.row, 1);
        else atomicAdd(nl_cnt + sl.row, 1);
    }
}

__global__ void plan_fill(ShareTables t, int32_t n_slots, const int32_t* row_ptr, const int32_t* nl_row_ptr,
                          int32_t* fill, int32_t* nl_fill, int32_t* col, int32_t* pos_slot,
                          int64_t* nl_col, int32_t* nl_pos_slot) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_slots; k += gridDim.x * blockDim.x) {
        const Slot sl = decode_slot(t, k);
        if (sl.kind == K_INVALID) continue;
        if (sl.colg >= t.lo && sl.colg < t.hi) {
            const int32_t pos = row_ptr[sl.row] + atomicAdd(fill + sl.row, 1);
            col[pos] = (int32_t)(sl.colg - t.lo);
            pos_slot[pos] = k;
        } else {
            const int32_t pos = nl_row_ptr[sl.row] + atomicAdd(nl_fill + sl.row, 1);
            nl_col[pos] = sl.colg;
            nl_pos_slot[pos] = k;
        }
    }
}

// insertion sort of each row's (column, slot) pairs by column; a repeated
// column is a duplicate matrix entry
template <typename C>
__global__ void plan_sort_rows(int32_t n_rows, const int32_t* row_ptr, C* col, int32_t* pos_slot,
                               uint32_t* flags) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_rows; i += gridDim.x * blockDim.x) {
        const int32_t a = row_ptr[i], b = row_ptr[i + 1];
        for (int32_t j = a + 1; j < b; ++j) {
            const C cj = col[j];
            const int32_t sj = pos_slot[j];
            int32_t m = j;
            while (m > a && col[m - 1] > cj) {
                col[m] = col[m - 1];
                pos_slot[m] = pos_slot[m - 1];
                --m;
            }
            col[m] = cj;
            pos_slot[m] = sj;
        }
        for (int32_t j = a + 1; j < b; ++j)
            if (col[j] == col[j - 1]) atomicOr(flags, (uint32_t)FLAG_MESH_DUP);
    }
}

__global__ void plan_perm(int32_t n_pos, int32_t pos_base, const int32_t* pos_slot, int32_t* perm) {
    for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_pos; j += gridDim.x * blockDim.x)
        perm[pos_slot[j]] = pos_base + j;
}

// interface pairing: a local coupling (row i, column j) from rank p must meet
// an interface slot of the partner rank at (j, i)
__global__ void plan_pair(ShareTables t, int32_t n_iface, const int32_t* row_ptr, const int32_t* col,
                          const int32_t* pos_slot, int32_t* partner) {
    for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n_iface; e += gridDim.x * blockDim.x) {
        const int32_t s = find_block(t.iface_off, t.alpha, e);
        const int32_t nc = t.row0[s + 1] - t.row0[s];
        const int32_t k = t.slot_off[s] + nc + 2 * t.nf[s] + (e - t.iface_off[s]);
        const Slot sl = decode_slot(t, k);
        partner[e] = -1;
        if (sl.kind != K_IFACE || !(sl.colg >= t.lo && sl.colg < t.hi)) continue;
        const int32_t j = (int32_t)(sl.colg - t.lo);
        int32_t a = row_ptr[j], b = row_ptr[j + 1];
        while (a < b) {  // lower bound of column sl.row in row j
            const int32_t m = (a + b) >> 1;
            if (col[m] < sl.row) a = m + 1; else b = m;
        }
        bool ok = false;
        if (a < row_ptr[j + 1] && col[a] == sl.row) {
            const int32_t k2 = pos_slot[a];
            const int32_t s2 = find_block(t.slot_off, t.alpha, k2);
            const int32_t nc2 = t.row0[s2 + 1] - t.row0[s2];
            ok = (k2 - t.slot_off[s2]) >= nc2 + 2 * t.nf[s2];
            if (ok) partner[e] = k2;
        }
        if (!ok) atomicOr(t.flags, (uint32_t)FLAG_MESH_UNPAIRED);
    }
}

// ---- exclusive scan of int32 counts: out[0..n] with out[n] = total --------
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = SCAN_BLOCK * SCAN_ITEMS;

__global__ void scan_reduce(const int32_t* in, int64_t n, int32_t* block_sums) {
    __shared__ int32_t red[SCAN_BLOCK / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    int32_t v = 0;
    for (int i = threadIdx.x; i < SCAN_CHUNK; i += SCAN_BLOCK)
        if (base + i < n) v += in[base + i];
    const int32_t s = block_sum<int32_t, SCAN_BLOCK>(v, red);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s;
}

// one block: exclusive scan of block_sums[0..nb) in place, total into [nb]
__global__ void scan_top(int32_t* block_sums, int32_t nb) {
    __shared__ int32_t wtot[1024 / 64];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t base = 0; base < nb; base += 1024) {
        const int32_t i = base + threadIdx.x;
        const int32_t v = i < nb ? block_sums[i] : 0;
        const int32_t inc = wave_incl_scan(v);
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        if (lane == 63) wtot[w] = inc;
        __syncthreads();
        int32_t woff = 0;
        for (int q = 0; q < w; ++q) woff += wtot[q];
        const int32_t c = carry;
        if (i < nb) block_sums[i] = c + woff + inc - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry = c + woff + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sums[nb] = carry;
}

__global__ void scan_down(const int32_t* in, int64_t n, const int32_t* block_sums, int32_t nb, int32_t* out) {
    __shared__ int32_t wtot[SCAN_BLOCK / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t tot = 0;
#pragma unroll
    for (int u = 0; u < SCAN_ITEMS; ++u) {
        v[u] = (base + u < n) ? in[base + u] : 0;
        tot += v[u];
    }
    const int32_t inc = wave_incl_scan(tot);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 63) wtot[w] = inc;
    __syncthreads();
    int32_t run = block_sums[blockIdx.x] + inc - tot;
    for (int q = 0; q < w; ++q) run += wtot[q];
#pragma unroll
    for (int u = 0; u < SCAN_ITEMS; ++u) {
        if (base + u < n) out[base + u] = run;
        run += v[u];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = block_sums[nb];
}

int exclusive_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* total, hipStream_t s) {
    const int32_t nb = (int32_t)((n + SCAN_CHUNK - 1) / SCAN_CHUNK);
    int32_t* sums = nullptr;
    RP_HIP_TRY(hipMalloc(&sums, sizeof(int32_t) * (nb + 1)));
    if (nb > 0) hipLaunchKernelGGL(scan_reduce, dim3(nb), dim3(SCAN_BLOCK), 0, s, in, n, sums);
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, s, sums, nb);
    hipLaunchKernelGGL(scan_down, dim3(nb > 0 ? nb : 1), dim3(SCAN_BLOCK), 0, s, in, n, sums, nb, out);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(total, sums + nb, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(sums);
    if (e != hipSuccess) {
        set_error("scan failed: %s", hipGetErrorString(e));
        return RP_ERR_HIP;
    }
    return RP_OK;
}

// SpMV x windows: sample the share's internal faces.  The diagonal window is
// used when at least a tenth of them couple cells at most XW_HALF apart in
// the rank's numbering; every |neighbour - owner| offset beyond that which
// a tenth of the faces share (at most two, most frequent first) gets a pair
// of windows at +-d.  Interface couplings are not counted: they leave the
// rank's numbering.
void detect_windows(rp_plan* p, const std::vector<int32_t>& owner, const std::vector<int32_t>& nbr) {
    p->xw_found = -1;
    p->xw_mode = -1;
    const size_t nf = owner.size();
    if (nf == 0) return;
    const size_t step = std::max<size_t>(1, nf / 262144);
    std::unordered_map<int64_t, int64_t> far;
    int64_t samples = 0, near = 0;
    for (size_t f = 0; f < nf; f += step) {
        const int64_t d = std::llabs((int64_t)nbr[f] - (int64_t)owner[f]);
        ++samples;
        if (d <= XW_HALF) ++near;
        else ++far[d];
    }
    if (10 * near < samples) return;
    p->xw_found = 0;
    for (int k = 0; k < 2; ++k) {
        int64_t best = 0, best_n = 0;
        for (const auto& kv : far)
            if (kv.second > best_n || (kv.second == best_n && kv.first < best)) {
                best = kv.first;
                best_n = kv.second;
            }
        if (10 * best_n < samples || best > INT32_MAX / 2) break;
        p->xw_d[k] = (int32_t)best;
        p->xw_found = k + 1;
        far.erase(best);
    }
}

int grid_for(int64_t n, int block = 256) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

template <typename T>
int upload(T** dst, const T* src, size_t count) {
    RP_HIP_TRY(hipMalloc(dst, sizeof(T) * (count > 0 ? count : 1)));
    if (count) RP_HIP_TRY(hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice));
    return RP_OK;
}

struct TempFree {
    std::vector<void*> ptrs;
    ~TempFree() {
        for (void* q : ptrs) (void)hipFree(q);
    }
};

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// offset-coded SpMV index (the form is described in spmv.hpp)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int32_t block_min_i32(int32_t v, int32_t* red) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    __syncthreads();  // red free from the previous call
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int32_t r = red[0];
    for (int w = 1; w < SPMV_BLOCK / 64; ++w) r = min(r, red[w]);
    return r;
}

// One block per group of SPMV_BLOCK rows (columns already sorted per row).
// The distinct offsets col - row of the group are found smallest first, one
// block-wide minimum per offset; a group with more than GOI_KMAX of them, or
// whose aligned value packs (2 doubles, 4 floats) would not fit SPMV_CAP
// elements, stays CSR (k = 0).
__global__ void __launch_bounds__(SPMV_BLOCK)
goi_encode(int32_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
           int32_t* __restrict__ goi_k, int32_t* __restrict__ goi_off, uint16_t* __restrict__ goi_mask) {
    __shared__ int32_t red[SPMV_BLOCK / 64];
    __shared__ int32_t tab[GOI_KMAX];
    const int32_t g = blockIdx.x, t = threadIdx.x;
    const int32_t r0 = g * SPMV_BLOCK, nr = min(SPMV_BLOCK, n - r0), i = r0 + t;
    int32_t rs = 0, re = 0;
    if (t < nr) {
        rs = row_ptr[i];
        re = row_ptr[i + 1];
    }
    const int32_t base = row_ptr[r0], end = row_ptr[r0 + nr];
    const int32_t npairs = (end - (base & ~1) + 1) >> 1;
    const int32_t nquads = (end - (base & ~3) + 3) >> 2;
    // offsets lie in (-n, n); INT32_MAX stands for "no further offset"
    int32_t ptr = rs, K = 0, cur = 0;
    bool over = npairs > SPMV_CAP / 2 || nquads > SPMV_CAP / 4;
    for (int round = 0; !over && round <= GOI_KMAX; ++round) {
        if (round > 0)
            while (ptr < re && col[ptr] - i <= cur) ++ptr;  // a row's offsets ascend with its columns
        const int32_t mn = block_min_i32(ptr < re ? col[ptr] - i : INT32_MAX, red);
        if (mn == INT32_MAX) break;
        if (round == GOI_KMAX) {
            over = true;
            break;
        }
        if (t == 0) tab[round] = mn;
        cur = mn;
        K = round + 1;
    }
    __syncthreads();  // tab complete
    if (over) K = 0;
    if (t < nr) {
        uint32_t m = 0;
        if (K > 0) {
            int32_t j = 0;
            for (int32_t e = rs; e < re; ++e) {
                const int32_t o = col[e] - i;
                while (j < K && tab[j] != o) ++j;  // every offset of the row is in tab
                if (j < K) m |= 1u << j;
            }
        }
        goi_mask[i] = (uint16_t)m;
    }
    if (t == 0) goi_k[g] = K;
    if (t < GOI_KMAX) goi_off[(int64_t)g * GOI_KMAX + t] = t < K ? tab[t] : 0;
}

// out[g] = k of group g, out[ng + g] = row_ptr[g * SPMV_BLOCK], out[2 ng] = row_ptr[n]
__global__ void goi_summary(int32_t n, int32_t ng, const int32_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ goi_k, int32_t* __restrict__ out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ng) {
        out[g] = goi_k[g];
        out[ng + g] = row_ptr[g * SPMV_BLOCK];
    }
    if (g == 0) out[2 * (int64_t)ng] = row_ptr[n];
}

// Build the coded index and count what it covers (n_groups, coded_groups,
// coded_rows, coded_nnz).
int goi_build(rp_plan* p, hipStream_t s) {
    const int64_t n = p->n_rows;
    const int64_t ng = (n + SPMV_BLOCK - 1) / SPMV_BLOCK;
    p->n_groups = ng;
    p->coded_groups = p->coded_rows = p->coded_nnz = 0;
    RP_HIP_TRY(hipMalloc(&p->d_goi_k, sizeof(int32_t) * (ng > 0 ? ng : 1)));
    RP_HIP_TRY(hipMalloc(&p->d_goi_off, sizeof(int32_t) * GOI_KMAX * (ng > 0 ? ng : 1)));
    RP_HIP_TRY(hipMalloc(&p->d_goi_mask, sizeof(uint16_t) * (n > 0 ? n : 1)));
    if (ng == 0) return RP_OK;
    hipLaunchKernelGGL(goi_encode, dim3((uint32_t)ng), dim3(SPMV_BLOCK), 0, s, (int32_t)n, p->d_row_ptr,
                       p->d_col, p->d_goi_k, p->d_goi_off, p->d_goi_mask);
    RP_HIP_TRY(hipGetLastError());
    // per group: k and the first entry (row_ptr at every SPMV_BLOCK-th row),
    // gathered on the device and copied back in one piece
    int32_t* d_sum = nullptr;
    RP_HIP_TRY(hipMalloc(&d_sum, sizeof(int32_t) * (2 * ng + 1)));
    std::vector<int32_t> h(2 * ng + 1);
    hipLaunchKernelGGL(goi_summary, dim3((uint32_t)((ng + 255) / 256)), dim3(256), 0, s, (int32_t)n, (int32_t)ng,
                       p->d_row_ptr, p->d_goi_k, d_sum);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d_sum, sizeof(int32_t) * (2 * ng + 1), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_sum);
    RP_HIP_TRY(e);
    const int32_t* k = h.data();
    const int32_t* start = h.data() + ng;
    for (int64_t g = 0; g < ng; ++g) {
        if (k[g] <= 0) continue;
        p->coded_groups += 1;
        p->coded_rows += std::min<int64_t>(SPMV_BLOCK, n - g * SPMV_BLOCK);
        p->coded_nnz += start[g + 1] - start[g];
    }
    return RP_OK;
}

}  // namespace

// exclusive scan of int32 counts for the other translation units:
// out[0..n] with out[n] = *total (read back to the host)
int scan_i32(const int32_t* in, int64_t n, int32_t* out, int32_t* total, hipStream_t s) {
    return exclusive_scan(in, n, out, total, s);
}

int plan_build(rp_plan* p, const rp_rank_desc* share) {
    const int32_t A = p->alpha;
    hipStream_t s = nullptr;
    TempFree tmp;

    // concatenated addressing of the share (host staging, then one upload each)
    std::vector<int32_t> face_off(A + 1, 0), owner, nbr, if_cell, if_rank, if_ncell;
    for (int32_t i = 0; i < A; ++i) face_off[i + 1] = face_off[i] + share[i].n_faces;
    owner.resize(face_off[A]);
    nbr.resize(face_off[A]);
    if_cell.resize(p->iface_off[A]);
    if_rank.resize(p->iface_off[A]);
    if_ncell.resize(p->iface_off[A]);
    for (int32_t i = 0; i < A; ++i) {
        const rp_rank_desc& d = share[i];
        std::copy(d.owner, d.owner + d.n_faces, owner.begin() + face_off[i]);
        std::copy(d.neighbour, d.neighbour + d.n_faces, nbr.begin() + face_off[i]);
        std::copy(d.iface_cell, d.iface_cell + d.n_iface, if_cell.begin() + p->iface_off[i]);
        std::copy(d.iface_nbr_rank, d.iface_nbr_rank + d.n_iface, if_rank.begin() + p->iface_off[i]);
        std::copy(d.iface_nbr_cell, d.iface_nbr_cell + d.n_iface, if_ncell.begin() + p->iface_off[i]);
    }

    int32_t *d_face_off = nullptr, *d_owner = nullptr, *d_nbr = nullptr;
    int32_t *d_if_cell = nullptr, *d_if_rank = nullptr, *d_if_ncell = nullptr;
    int64_t* d_off_all = nullptr;
    int rc;
    if ((rc = upload(&p->d_slot_off, p->slot_off.data(), A + 1))) return rc;
    if ((rc = upload(&p->d_row0, p->row0.data(), A + 1))) return rc;
    if ((rc = upload(&p->d_nf, p->n_faces.data(), A))) return rc;
    if ((rc = upload(&p->d_iface_off, p->iface_off.data(), A + 1))) return rc;
    detect_windows(p, owner, nbr);
    if ((rc = upload(&d_face_off, face_off.data(), A + 1))) return rc;
    p->d_face_off = d_face_off;
    // the face addressing stays on the device for the value gradient
    if ((rc = upload(&d_owner, owner.data(), owner.size()))) return rc;
    p->d_owner = d_owner;
    if ((rc = upload(&d_nbr, nbr.data(), nbr.size()))) return rc;
    p->d_nbr = d_nbr;
    if ((rc = upload(&d_if_cell, if_cell.data(), if_cell.size()))) return rc;
    tmp.ptrs.push_back(d_if_cell);
    if ((rc = upload(&d_if_rank, if_rank.data(), if_rank.size()))) return rc;
    tmp.ptrs.push_back(d_if_rank);
    if ((rc = upload(&d_if_ncell, if_ncell.data(), if_ncell.size()))) return rc;
    tmp.ptrs.push_back(d_if_ncell);
    if ((rc = upload(&d_off_all, p->off_all.data(), p->off_all.size()))) return rc;
    tmp.ptrs.push_back(d_off_all);
    RP_HIP_TRY(hipMalloc(&p->d_flags, sizeof(uint32_t) * 2));
    RP_HIP_TRY(hipMemset(p->d_flags, 0, sizeof(uint32_t) * 2));
    owner.clear(); owner.shrink_to_fit();
    nbr.clear(); nbr.shrink_to_fit();

    ShareTables t;
    t.slot_off = p->d_slot_off; t.row0 = p->d_row0; t.nf = p->d_nf; t.face_off = d_face_off;
    t.owner = d_owner; t.nbr = d_nbr; t.iface_off = p->d_iface_off;
    t.if_cell = d_if_cell; t.if_rank = d_if_rank; t.if_ncell = d_if_ncell; t.off_all = d_off_all;
    t.flags = p->d_flags;
    t.lo = p->off_all[p->first];
    t.hi = p->off_all[p->first + A];
    t.alpha = A; t.first = p->first; t.n_ranks_total = p->n_ranks_total;

    const int64_t n = p->n_rows;
    const int32_t ns = (int32_t)p->n_slots;
    int32_t *cnt = nullptr, *nl_cnt = nullptr;
    RP_HIP_TRY(hipMalloc(&cnt, sizeof(int32_t) * (n + 1)));
    tmp.ptrs.push_back(cnt);
    RP_HIP_TRY(hipMalloc(&nl_cnt, sizeof(int32_t) * (n + 1)));
    tmp.ptrs.push_back(nl_cnt);
    RP_HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (n + 1), s));
    RP_HIP_TRY(hipMemsetAsync(nl_cnt, 0, sizeof(int32_t) * (n + 1), s));
    hipLaunchKernelGGL(plan_count, dim3(grid_for(ns)), dim3(256), 0, s, t, ns, cnt, nl_cnt);
    RP_HIP_TRY(hipGetLastError());

    uint32_t flags = 0;
    RP_HIP_TRY(hipMemcpyAsync(&flags, p->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    if (flags) {
        set_error("invalid LDU addressing in the share (flags 0x%x: %s%s)", flags,
                  (flags & FLAG_MESH_RANGE) ? "index out of range " : "",
                  (flags & FLAG_MESH_SELF) ? "owner == neighbour or interface to own rank" : "");
        return RP_ERR_MESH;
    }

    RP_HIP_TRY(hipMalloc(&p->d_row_ptr, sizeof(int32_t) * (n + 1)));
    RP_HIP_TRY(hipMalloc(&p->d_nl_row_ptr, sizeof(int32_t) * (n + 1)));
    int32_t nnz = 0, nnz_nl = 0;
    if ((rc = exclusive_scan(cnt, n, p->d_row_ptr, &nnz, s))) return rc;
    if ((rc = exclusive_scan(nl_cnt, n, p->d_nl_row_ptr, &nnz_nl, s))) return rc;
    if ((int64_t)nnz + nnz_nl != p->n_slots) {
        set_error("internal: counted %d + %d entries for %lld slots", nnz, nnz_nl, (long long)p->n_slots);
        return RP_ERR_HIP;
    }
    p->nnz = nnz;
    p->nnz_nl = nnz_nl;

    RP_HIP_TRY(hipMalloc(&p->d_col, sizeof(int32_t) * ((size_t)nnz + SPMV_PAD)));
    RP_HIP_TRY(hipMemsetAsync(p->d_col + nnz, 0, sizeof(int32_t) * SPMV_PAD, s));
    RP_HIP_TRY(hipMalloc(&p->d_perm_inv, sizeof(int32_t) * (p->n_slots > 0 ? p->n_slots : 1)));
    RP_HIP_TRY(hipMalloc(&p->d_perm, sizeof(int32_t) * (p->n_slots > 0 ? p->n_slots : 1)));
    RP_HIP_TRY(hipMalloc(&p->d_nl_col, sizeof(int64_t) * (nnz_nl > 0 ? nnz_nl : 1)));
    RP_HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (n + 1), s));
    RP_HIP_TRY(hipMemsetAsync(nl_cnt, 0, sizeof(int32_t) * (n + 1), s));
    hipLaunchKernelGGL(plan_fill, dim3(grid_for(ns)), dim3(256), 0, s, t, ns, p->d_row_ptr, p->d_nl_row_ptr,
                       cnt, nl_cnt, p->d_col, p->d_perm_inv, p->d_nl_col, p->d_perm_inv + nnz);
    RP_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(plan_sort_rows<int32_t>, dim3(grid_for(n)), dim3(256), 0, s, (int32_t)n, p->d_row_ptr,
                       p->d_col, p->d_perm_inv, p->d_flags);
    if (nnz_nl > 0)
        hipLaunchKernelGGL(plan_sort_rows<int64_t>, dim3(grid_for(n)), dim3(256), 0, s, (int32_t)n,
                           p->d_nl_row_ptr, p->d_nl_col, p->d_perm_inv + nnz, p->d_flags);
    hipLaunchKernelGGL(plan_perm, dim3(grid_for(nnz)), dim3(256), 0, s, nnz, 0, p->d_perm_inv, p->d_perm);
    if (nnz_nl > 0)
        hipLaunchKernelGGL(plan_perm, dim3(grid_for(nnz_nl)), dim3(256), 0, s, nnz_nl, nnz, p->d_perm_inv + nnz,
                           p->d_perm);
    RP_HIP_TRY(hipGetLastError());

    const int32_t ni = p->iface_off[A];
    p->n_iface_share = ni;
    RP_HIP_TRY(hipMalloc(&p->d_iface_partner, sizeof(int32_t) * (ni > 0 ? ni : 1)));
    if (ni > 0) {
        hipLaunchKernelGGL(plan_pair, dim3(grid_for(ni)), dim3(256), 0, s, t, ni, p->d_row_ptr, p->d_col,
                           p->d_perm_inv, p->d_iface_partner);
        RP_HIP_TRY(hipGetLastError());
    }
    RP_HIP_TRY(hipMemcpyAsync(&flags, p->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    if (flags) {
        set_error("invalid LDU addressing in the share (flags 0x%x: %s%s)", flags,
                  (flags & FLAG_MESH_DUP) ? "a matrix entry is addressed twice " : "",
                  (flags & FLAG_MESH_UNPAIRED) ? "an interface coupling has no partner" : "");
        return RP_ERR_MESH;
    }
    return goi_build(p, s);
}

}  // namespace rp

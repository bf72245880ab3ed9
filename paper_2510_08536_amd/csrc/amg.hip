// Aggregation multigrid preconditioner (rp_solve_opts.precond =
// RP_PRECOND_AMG), the multigrid option of the outlook in Sec. 5.
//
// Hierarchy (built once from the values at hand, rp_plan_amg_setup or the
// first solve that asks for it; the aggregates and patterns are then kept,
// and every later value update refreshes only the coarse values):
//  * pairwise matching in rounds on the negative couplings: every unmatched
//    row picks its strongest coupling to an unmatched row, rows that picked
//    each other pair up; a row left over joins the pair of its strongest
//    coupling to a matched row, else stays alone.  Strength: the value's
//    magnitude, ties broken by a hash of the row pair (MurmurHash3's 32-bit
//    finaliser), then by the smaller pair.  Aggregates are numbered by their
//    leaders (a pair's smaller row), ascending.
//  * Galerkin coarse matrix A_c = P^T A P, P the aggregate indicator: each
//    coarse entry sums its fine entries in ascending fine CSR position.  The
//    plan keeps, per coarse entry, the list of those positions, so a value
//    refresh is a gather-sum through a fixed map (like the update by P).
//  * coarsest level (at most AMG_COARSE_MAX rows): dense Gauss-Jordan
//    inverse without pivoting in the textbook order, one workgroup.
// V-cycle y = V_l(r): even levels smooth with one damped-Jacobi sweep from
// zero, restrict the residual, add the prolonged coarse correction and
// smooth again; odd levels only restrict and prolong (two pairwise passes
// per smoothed level); the coarsest level multiplies by the dense inverse.
// Every product and sum is one rounding in the order the definition states
// (row sums in column order, aggregate sums over the members ascending), so
// the hierarchy and one V-cycle are bit-exact against the serial definition.
// The levels from the first one with at most AMG_TAIL_ROWS rows down run in
// one workgroup (amg_tail), with the same operations in the same order.
//
// Setup runs on the device: matching rounds (the host reads one counter per
// round), scans for the numbering, per-coarse-row key lists (aggregate of the
// column, fine position) sorted in place for the patterns and the
// contribution lists.
#include "spmv.hpp"

namespace rp {

int scan_i32(const int32_t* in, int64_t n, int32_t* out, int32_t* total, hipStream_t s);

namespace {

constexpr int AB = 256;   // threads per block of the setup and vector kernels

int grid_of(int64_t n) {
    int64_t g = (n + AB - 1) / AB;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 16384));
}

// ---- coupling strength -----------------------------------------------------
__device__ __forceinline__ uint32_t fmix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return x;
}

// strongest negative coupling of row i to a row whose matched state is
// `matched`; -1 if none.  The comparison is one boolean expression and the
// running best is updated by selects: the form with nested branches was
// compiled (hipcc, gfx950) into code that kept the first candidate's weight.
__device__ int32_t strongest(int32_t i, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                             const double* __restrict__ val, const int32_t* __restrict__ mate, bool matched) {
    int32_t best = -1, blo = 0, bhi = 0;
    double bw = 0.0;
    uint32_t bh = 0u;
    for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        const int32_t j = col[p];
        const double a = val[p];
        const bool cand = j != i && a < 0.0 && ((mate[j] >= 0) == matched);
        const double w = -a;
        const int32_t lo = min(i, j), hi = max(i, j);
        const uint32_t h = fmix32((uint32_t)lo * 0x9E3779B1u + (uint32_t)hi);
        const bool better = (w > bw) | ((w == bw) & ((h > bh) | ((h == bh) & ((lo < blo) | ((lo == blo) & (hi < bhi))))));
        const bool take = cand & ((best < 0) | better);
        best = take ? j : best;
        bw = take ? w : bw;
        bh = take ? h : bh;
        blo = take ? lo : blo;
        bhi = take ? hi : bhi;
    }
    return best;
}

// ---- setup kernels -----------------------------------------------------------
__global__ void amg_fill(int32_t n, int32_t v, int32_t* a) {
    for (int32_t i = blockIdx.x * AB + threadIdx.x; i < n; i += gridDim.x * AB) a[i] = v;
}

__global__ void __launch_bounds__(AB)
amg_pick(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val, const int32_t* mate,
         int32_t* pick) {
    for (int32_t i = blockIdx.x * AB + threadIdx.x; i < n; i += gridDim.x * AB)
        pick[i] = mate[i] >= 0 ? -1 : strongest(i, row_ptr, col, val, mate, false);
}

// rows that picked each other pair up; count[0] += pairs (two rows each)
__global__ void __launch_bounds__(AB)
amg_pair(int32_t n, const int32_t* pick, int32_t* mate, uint32_t* count) {
    uint32_t c = 0;
    for (int32_t i = blockIdx.x * AB + threadIdx.x; i < n; i += gridDim.x * AB) {
        const int32_t j = pick[i];
        if (j >= 0 && pick[j] == i) {
            mate[i] = j;
            ++c;
        }
    }
    if (c) atomicAdd(count, c);
}

__global__ void __launch_bounds__(AB)
amg_leader(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val, const int32_t* mate,
           int32_t* leader, int32_t* is_leader) {
    for (int32_t i = blockIdx.x * AB + threadIdx.x; i < n; i += gridDim.x * AB) {
        int32_t l;
        if (mate[i] >= 0) {
            l = min(i, mate[i]);
        } else {
            const int32_t j = strongest(i, row_ptr, col, val, mate, true);
            l = j >= 0 ? min(j, mate[j]) : i;
        }
        leader[i] = l;
        is_leader[i] = l == i ? 1 : 0;
    }
}

// agg[i] = number of leaders below leader[i]; members counted per aggregate
__global__ void __launch_bounds__(AB)
amg_number(int32_t n, const int32_t* leader, const int32_t* lead_id, int32_t* agg, int32_t* cnt) {
    for (int32_t i = blockIdx.x * AB + threadIdx.x; i < n; i += gridDim.x * AB) {
        const int32_t a = lead_id[leader[i]];
        agg[i] = a;
        atomicAdd(cnt + a, 1);
    }
}

__global__ void __launch_bounds__(AB)
amg_members(int32_t n, const int32_t* agg, const int32_t* mem_ptr, int32_t* fill, int32_t* mem) {
    for (int32_t i = blockIdx.x * AB + threadIdx.x; i < n; i += gridDim.x * AB) {
        const int32_t a = agg[i];
        mem[mem_ptr[a] + atomicAdd(fill + a, 1)] = i;
    }
}

// per aggregate: members ascending (insertion sort, aggregates are small);
// keys of the coarse row counted
__global__ void __launch_bounds__(AB)
amg_sort_members(int32_t nc, const int32_t* mem_ptr, int32_t* mem, const int32_t* row_ptr, int32_t* kcnt) {
    for (int32_t I = blockIdx.x * AB + threadIdx.x; I < nc; I += gridDim.x * AB) {
        const int32_t a0 = mem_ptr[I], a1 = mem_ptr[I + 1];
        int32_t k = 0;
        for (int32_t a = a0; a < a1; ++a) {
            const int32_t v = mem[a];
            int32_t b = a;
            while (b > a0 && mem[b - 1] > v) {
                mem[b] = mem[b - 1];
                --b;
            }
            mem[b] = v;
            k += row_ptr[v + 1] - row_ptr[v];
        }
        kcnt[I] = k;
    }
}

// keys (aggregate of the column << 32 | fine position) of coarse row I,
// sorted; the number of distinct coarse columns into ucnt[I]
__global__ void __launch_bounds__(AB)
amg_keys(int32_t nc, const int32_t* mem_ptr, const int32_t* mem, const int32_t* row_ptr, const int32_t* col,
         const int32_t* agg, const int32_t* kstart, uint64_t* keys, int32_t* ucnt) {
    for (int32_t I = blockIdx.x * AB + threadIdx.x; I < nc; I += gridDim.x * AB) {
        const int32_t k0 = kstart[I];
        int32_t k = k0;
        for (int32_t m = mem_ptr[I]; m < mem_ptr[I + 1]; ++m) {
            const int32_t i = mem[m];
            for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                keys[k++] = ((uint64_t)(uint32_t)agg[col[p]] << 32) | (uint32_t)p;
        }
        for (int32_t a = k0 + 1; a < k; ++a) {
            const uint64_t v = keys[a];
            int32_t b = a;
            while (b > k0 && keys[b - 1] > v) {
                keys[b] = keys[b - 1];
                --b;
            }
            keys[b] = v;
        }
        int32_t u = 0;
        for (int32_t a = k0; a < k; ++a)
            if (a == k0 || (keys[a] >> 32) != (keys[a - 1] >> 32)) ++u;
        ucnt[I] = u;
    }
}

// coarse columns, diagonal positions, contribution ranges and positions
__global__ void __launch_bounds__(AB)
amg_cfill(int32_t nc, const int32_t* kstart, const uint64_t* keys, const int32_t* c_row_ptr, int32_t* c_col,
          int32_t* c_diag, int32_t* cptr, int32_t* cpos) {
    for (int32_t I = blockIdx.x * AB + threadIdx.x; I < nc; I += gridDim.x * AB) {
        int32_t e = c_row_ptr[I];
        int32_t diag = -1;
        for (int32_t a = kstart[I]; a < kstart[I + 1]; ++a) {
            const int32_t J = (int32_t)(keys[a] >> 32);
            if (a == kstart[I] || J != (int32_t)(keys[a - 1] >> 32)) {
                cptr[e] = a;
                c_col[e] = J;
                if (J == I) diag = e;
                ++e;
            }
            cpos[a] = (int32_t)(keys[a] & 0xFFFFFFFFu);
        }
        c_diag[I] = diag;
        if (I == nc - 1) cptr[e] = kstart[nc];
    }
}

// ---- value refresh -----------------------------------------------------------
__global__ void __launch_bounds__(AB)
amg_gvals(int32_t nnz_c, const int32_t* cptr, const int32_t* cpos, const double* fine, double* c64, float* c32) {
#pragma clang fp contract(off)
    for (int32_t e = blockIdx.x * AB + threadIdx.x; e < nnz_c; e += gridDim.x * AB) {
        double s = 0.0;
        for (int32_t t = cptr[e]; t < cptr[e + 1]; ++t) s += fine[cpos[t]];
        c64[e] = s;
        c32[e] = (float)s;
    }
}

__global__ void __launch_bounds__(AB)
amg_gdiag(int32_t nc, const int32_t* c_diag, const double* c64, double* dinv64, float* dinv32, uint32_t* flag) {
    for (int32_t I = blockIdx.x * AB + threadIdx.x; I < nc; I += gridDim.x * AB) {
        const int32_t e = c_diag[I];
        const double d = e >= 0 ? c64[e] : 0.0;
        if (!(d > 0.0) || !isfinite(d)) atomicOr(flag, 1u);
        const double v = 1.0 / d;
        dinv64[I] = v;
        dinv32[I] = (float)v;
    }
}

// dense Gauss-Jordan inverse of the n x n coarsest matrix (n <= AMG_COARSE_MAX),
// one workgroup: pivot row divided, multipliers of column k read, then every
// other row updated; the same single roundings in the same order as the
// serial elimination.  W: n*n work, Z: the inverse.
constexpr int GJ_THREADS = 1024;

__global__ void __launch_bounds__(GJ_THREADS)
amg_dense_inverse(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val, double* W, double* Z,
                  float* Z32, uint32_t* flag) {
#pragma clang fp contract(off)
    __shared__ double f[AMG_COARSE_MAX];
    __shared__ double piv_s;
    const int32_t t = threadIdx.x, nn = n * n;
    for (int32_t e = t; e < nn; e += GJ_THREADS) {
        W[e] = 0.0;
        Z[e] = (e / n == e % n) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int32_t i = t; i < n; i += GJ_THREADS)
        for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) W[i * n + col[p]] = val[p];
    __syncthreads();
    for (int32_t k = 0; k < n; ++k) {
        if (t == 0) piv_s = W[k * n + k];
        __syncthreads();
        const double piv = piv_s;
        if (!(piv > 0.0) || !isfinite(piv)) {
            if (t == 0) atomicOr(flag, 2u);
            return;
        }
        for (int32_t j = t; j < n; j += GJ_THREADS) {
            W[k * n + j] = W[k * n + j] / piv;
            Z[k * n + j] = Z[k * n + j] / piv;
        }
        __syncthreads();
        for (int32_t i = t; i < n; i += GJ_THREADS) f[i] = W[i * n + k];
        __syncthreads();
        for (int32_t e = t; e < nn; e += GJ_THREADS) {
            const int32_t i = e / n, j = e - i * n;
            if (i == k) continue;
            W[e] = W[e] - f[i] * W[k * n + j];
            Z[e] = Z[e] - f[i] * Z[k * n + j];
        }
        __syncthreads();
    }
    for (int32_t e = t; e < nn; e += GJ_THREADS) Z32[e] = (float)Z[e];
}

// ---- V-cycle kernels -----------------------------------------------------------
// gate: the solve's K2-written iteration word; < 0 means K2 did no update
// this iteration and the cycle's result is not used, so every kernel returns

// x = omega (dinv r)
template <typename T>
__global__ void __launch_bounds__(AB)
amg_pre(int32_t n, const T* __restrict__ r, const T* __restrict__ dinv, T* __restrict__ x, T omega,
        const int32_t* gate) {
#pragma clang fp contract(off)
    if (gate && *gate < 0) return;
    for (int32_t i = blockIdx.x * AB + threadIdx.x; i < n; i += gridDim.x * AB) x[i] = omega * (dinv[i] * r[i]);
}

// t = r - A x
template <typename T>
__global__ void __launch_bounds__(SPMV_BLOCK)
amg_resid(int32_t n, SpmvIdx ix, const T* __restrict__ val, const T* __restrict__ x, const T* __restrict__ r,
          T* __restrict__ t, const int32_t* gate) {
#pragma clang fp contract(off)
    __shared__ __align__(16) T lds[SPMV_CAP];
    __shared__ T xs[1];
    if (gate && *gate < 0) return;
    const XWin w{{0, 0}};
    GroupRange gr = block_groups(ix, n);
    for (int32_t g = gr.g0; g < gr.n_groups; g += gr.step) {
        const int32_t r0 = g * SPMV_BLOCK;
        const int32_t nr = min(SPMV_BLOCK, n - r0);
        const GroupRow<T> row = spmv_group_row<T, -1>(ix, val, x, n, g, nr, w, xs, lds, gr);
        if ((int32_t)threadIdx.x < nr) {
            const int32_t i = r0 + threadIdx.x;
            t[i] = r[i] - row.s;
        }
    }
}

// Coarse levels (plain CSR, 10 to 30 entries per row): one wavefront per
// block, chunks of CR consecutive rows (64, or 32 on levels with more than
// 12 entries per row).  The wave forms the chunk's products val * x together
// (coalesced over the entries, every load of a lane issued before the first
// product) into LDS, then each lane sums its row's products in column order
// from 0: the same single roundings as the serial row sum.  A chunk with
// more than WCAP entries is summed straight from memory, a lane per row.
constexpr int WB = 64;            // threads per block: one wavefront
constexpr int WCAP = 1024;        // staged products per chunk
constexpr int WU = WCAP / WB;     // loads per lane

template <typename T>
__device__ __forceinline__ T wave_row_sum(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                          const T* __restrict__ val, const T* __restrict__ x, int32_t r0,
                                          int32_t nr, T* prod) {
#pragma clang fp contract(off)
    const int32_t t = threadIdx.x;
    const int32_t e0 = row_ptr[r0], e1 = row_ptr[r0 + nr];
    T s = T(0);
    if (e1 - e0 <= WCAP) {
        int32_t cv[WU];
        T vv[WU], xv[WU];
#pragma unroll
        for (int u = 0; u < WU; ++u) {
            const int32_t e = e0 + t + u * WB;
            cv[u] = e < e1 ? col[e] : 0;
            vv[u] = e < e1 ? val[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < WU; ++u) xv[u] = (e0 + t + u * WB < e1) ? x[cv[u]] : T(0);
#pragma unroll
        for (int u = 0; u < WU; ++u) {
            const int32_t e = e0 + t + u * WB;
            if (e < e1) prod[e - e0] = vv[u] * xv[u];
        }
        __syncthreads();   // one wave: orders its LDS writes before the reads
        if (t < nr)
            for (int32_t e = row_ptr[r0 + t]; e < row_ptr[r0 + t + 1]; ++e) s += prod[e - e0];
        __syncthreads();   // prod is refilled by the next chunk
    } else if (t < nr) {
        for (int32_t e = row_ptr[r0 + t]; e < row_ptr[r0 + t + 1]; ++e) s += val[e] * x[col[e]];
    }
    return s;
}

// t = r - A x on a coarse level
template <typename T, int CR>
__global__ void __launch_bounds__(WB)
amg_csr_resid(int32_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
              const T* __restrict__ val, const T* __restrict__ x, const T* __restrict__ r, T* __restrict__ t,
              const int32_t* gate) {
#pragma clang fp contract(off)
    __shared__ T prod[WCAP];
    if (gate && *gate < 0) return;
    const int32_t nch = (n + CR - 1) / CR;
    for (int32_t c = xcd_block(); c < nch; c += gridDim.x) {
        const int32_t r0 = c * CR, nr = min(CR, n - r0);
        const T s = wave_row_sum<T>(row_ptr, col, val, x, r0, nr, prod);
        if ((int32_t)threadIdx.x < nr) {
            const int32_t i = r0 + threadIdx.x;
            t[i] = r[i] - s;
        }
    }
}

// y = x + omega (dinv (r - A x)) on a coarse level
template <typename T, int CR>
__global__ void __launch_bounds__(WB)
amg_csr_post(int32_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
             const T* __restrict__ val, const T* __restrict__ x, const T* __restrict__ r,
             const T* __restrict__ dinv, T omega, T* __restrict__ y, const int32_t* gate) {
#pragma clang fp contract(off)
    __shared__ T prod[WCAP];
    if (gate && *gate < 0) return;
    const int32_t nch = (n + CR - 1) / CR;
    for (int32_t c = xcd_block(); c < nch; c += gridDim.x) {
        const int32_t r0 = c * CR, nr = min(CR, n - r0);
        const T s = wave_row_sum<T>(row_ptr, col, val, x, r0, nr, prod);
        if ((int32_t)threadIdx.x < nr) {
            const int32_t i = r0 + threadIdx.x;
            y[i] = x[i] + omega * (dinv[i] * (r[i] - s));
        }
    }
}

// chunk rows of a level: 64, or 32 where rows average more than 12 entries
int chunk_rows(const AmgLevel& L) { return L.nnz > 12 * L.n ? 32 : 64; }

// grid of the chunked kernels: a multiple of 8 (xcd_block), one chunk per
// block up to 16384 blocks
int chunk_grid(int64_t n, int cr) {
    int64_t g = (n + cr - 1) / cr;
    g = ((g + N_XCD - 1) / N_XCD) * N_XCD;
    return (int)std::max<int64_t>(N_XCD, std::min<int64_t>(g, 16384));
}

// rc[I] = sum of v over the members of aggregate I, ascending
template <typename T>
__global__ void __launch_bounds__(AB)
amg_restrict(int32_t nc, const int32_t* __restrict__ mem_ptr, const int32_t* __restrict__ mem,
             const T* __restrict__ v, T* __restrict__ rc, const int32_t* gate) {
#pragma clang fp contract(off)
    if (gate && *gate < 0) return;
    constexpr int M = 8;   // aggregates up to M rows: every load issued first
    for (int32_t I = blockIdx.x * AB + threadIdx.x; I < nc; I += gridDim.x * AB) {
        const int32_t a0 = mem_ptr[I], a1 = mem_ptr[I + 1];
        T s = T(0);
        if (a1 - a0 <= M) {
            int32_t mi[M];
            T vv[M];
#pragma unroll
            for (int u = 0; u < M; ++u) mi[u] = a0 + u < a1 ? mem[a0 + u] : 0;
#pragma unroll
            for (int u = 0; u < M; ++u) vv[u] = a0 + u < a1 ? v[mi[u]] : T(0);
#pragma unroll
            for (int u = 0; u < M; ++u)
                if (a0 + u < a1) s += vv[u];
        } else {
            for (int32_t m = a0; m < a1; ++m) s += v[mem[m]];
        }
        rc[I] = s;
    }
}

// x += e[agg]  (ADD) or  y = e[agg]
template <typename T, bool ADD>
__global__ void __launch_bounds__(AB)
amg_prolong(int32_t n, const int32_t* __restrict__ agg, const T* __restrict__ e, T* __restrict__ y,
            const int32_t* gate) {
#pragma clang fp contract(off)
    if (gate && *gate < 0) return;
    for (int32_t i = blockIdx.x * AB + threadIdx.x; i < n; i += gridDim.x * AB)
        y[i] = ADD ? y[i] + e[agg[i]] : e[agg[i]];
}

// y = x + omega (dinv (r - A x)); PART: partials of (r, y) -> PART_RZ and,
// RR, of (r, r) -> PART_RR, one per block at xcd_block()
template <typename T, bool PART, bool RR>
__global__ void __launch_bounds__(SPMV_BLOCK)
amg_post(int32_t n, SpmvIdx ix, const T* __restrict__ val, const T* __restrict__ x, const T* __restrict__ r,
         const T* __restrict__ dinv, T omega, T* __restrict__ y, T* __restrict__ part, const int32_t* gate) {
#pragma clang fp contract(off)
    __shared__ __align__(16) T lds[SPMV_CAP];
    __shared__ T xs[1];
    __shared__ T red[SPMV_BLOCK / 64];
    if (gate && *gate < 0) return;
    const XWin w{{0, 0}};
    T prz = T(0), prr = T(0);
    GroupRange gr = block_groups(ix, n);
    for (int32_t g = gr.g0; g < gr.n_groups; g += gr.step) {
        const int32_t r0 = g * SPMV_BLOCK;
        const int32_t nr = min(SPMV_BLOCK, n - r0);
        const GroupRow<T> row = spmv_group_row<T, -1>(ix, val, x, n, g, nr, w, xs, lds, gr);
        if ((int32_t)threadIdx.x < nr) {
            const int32_t i = r0 + threadIdx.x;
            const T ri = r[i];
            const T yi = x[i] + omega * (dinv[i] * (ri - row.s));
            y[i] = yi;
            prz += ri * yi;
            prr += ri * ri;
        }
    }
    if (PART) {
        const T b1 = block_sum<T, SPMV_BLOCK>(prz, red);
        if (RR) {
            const T b2 = block_sum<T, SPMV_BLOCK>(prr, red);
            if (threadIdx.x == 0) part[PART_RR + xcd_block()] = b2;
        }
        if (threadIdx.x == 0) part[PART_RZ + xcd_block()] = b1;
    }
}

// y = Cinv r on the coarsest level (one block); PART as amg_post
template <typename T, bool PART, bool RR>
__global__ void __launch_bounds__(AB)
amg_coarse(int32_t n, const T* __restrict__ cinv, const T* __restrict__ r, T* __restrict__ y, T* __restrict__ part,
           int32_t n_part, const int32_t* gate) {
#pragma clang fp contract(off)
    __shared__ T rs[AMG_COARSE_MAX];
    __shared__ T red[AB / 64];
    if (gate && *gate < 0) return;
    for (int32_t j = threadIdx.x; j < n; j += AB) rs[j] = r[j];
    __syncthreads();
    T prz = T(0), prr = T(0);
    for (int32_t i = threadIdx.x; i < n; i += AB) {
        T s = T(0);
        for (int32_t j = 0; j < n; ++j) s += cinv[(int64_t)i * n + j] * rs[j];
        y[i] = s;
        prz += rs[i] * s;
        prr += rs[i] * rs[i];
    }
    if (PART) {
        // the solve sums n_part partials: this block's, then zeros
        const T b1 = block_sum<T, AB>(prz, red);
        const T b2 = RR ? block_sum<T, AB>(prr, red) : T(0);
        if (threadIdx.x == 0) {
            part[PART_RZ] = b1;
            if (RR) part[PART_RR] = b2;
        }
        for (int32_t q = 1 + threadIdx.x; q < n_part; q += AB) {
            part[PART_RZ + q] = T(0);
            if (RR) part[PART_RR + q] = T(0);
        }
    }
}

// ---------------------------------------------------------------------------
// The tail of the V-cycle: every level from the first one with at most
// AMG_TAIL_ROWS rows down to the coarsest, in one workgroup.  Each step is
// the corresponding kernel's above, row by row with the same operations in
// the same order (rows' products summed in column order from 0, members in
// ascending order, the coarsest inverse times r with j ascending), and the
// workgroup barrier stands where the level kernels had a launch boundary.
// On the small levels a launch costs more than its work.
// ---------------------------------------------------------------------------
constexpr int64_t AMG_TAIL_ROWS = RP_AMG_TAIL_ROWS;
constexpr int TB = 1024;   // threads of the tail workgroup

template <typename T>
struct TailLevel {
    int32_t n;
    const int32_t* row_ptr;
    const int32_t* col;
    const T* val;
    const T* dinv;
    const int32_t* agg;       // all tail levels but the coarsest
    const int32_t* mem_ptr;
    const int32_t* mem;
    T* v[4];                  // in, x, t, out (x and t on smoothed levels)
};

// row i of A x: U entries per trip, every load of a trip issued before its
// first product; the products are added in column order from 0
template <typename T>
__device__ __forceinline__ T tail_row_sum(const TailLevel<T>& L, const T* __restrict__ x, int32_t i) {
#pragma clang fp contract(off)
    constexpr int U = 8;
    T s = T(0);
    const int32_t e0 = L.row_ptr[i], e1 = L.row_ptr[i + 1];
    for (int32_t eb = e0; eb < e1; eb += U) {
        int32_t c[U];
        T v[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = eb + u < e1;
            c[u] = in ? L.col[eb + u] : 0;
            v[u] = in ? L.val[eb + u] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (eb + u < e1) s += v[u] * xv[u];
    }
    return s;
}

// y = V_lt(r) on levels lt .. last (lv[0] is level lt; r in lv[0].v[0], y
// to lv[0].v[3])
template <typename T>
__global__ void __launch_bounds__(TB)
amg_tail(int32_t lt, int32_t last, const TailLevel<T>* __restrict__ lv, const T* __restrict__ cinv, T omega,
         const int32_t* gate) {
#pragma clang fp contract(off)
    if (gate && *gate < 0) return;
    const int32_t t = threadIdx.x;
    for (int32_t l = lt; l < last; ++l) {
        const TailLevel<T>& L = lv[l - lt];
        const TailLevel<T>& C = lv[l - lt + 1];
        const T* r = L.v[0];
        const T* src = r;   // what restricts to the coarse level
        if (l % 2 == 0) {
            for (int32_t i = t; i < L.n; i += TB) L.v[1][i] = omega * (L.dinv[i] * r[i]);
            __syncthreads();
            for (int32_t i = t; i < L.n; i += TB) L.v[2][i] = r[i] - tail_row_sum(L, L.v[1], i);
            __syncthreads();
            src = L.v[2];
        }
        for (int32_t I = t; I < C.n; I += TB) {
            T s = T(0);
            for (int32_t m = L.mem_ptr[I]; m < L.mem_ptr[I + 1]; ++m) s += src[L.mem[m]];
            C.v[0][I] = s;
        }
        __syncthreads();
    }
    {
        const TailLevel<T>& L = lv[last - lt];
        const int32_t n = L.n;
        for (int32_t i = t; i < n; i += TB) {
            T s = T(0);
            for (int32_t j = 0; j < n; ++j) s += cinv[(int64_t)i * n + j] * L.v[0][j];
            L.v[3][i] = s;
        }
        __syncthreads();
    }
    for (int32_t l = last - 1; l >= lt; --l) {
        const TailLevel<T>& L = lv[l - lt];
        const T* e = lv[l - lt + 1].v[3];
        if (l % 2 == 1) {
            for (int32_t i = t; i < L.n; i += TB) L.v[3][i] = e[L.agg[i]];
        } else {
            T* x = L.v[1];
            for (int32_t i = t; i < L.n; i += TB) x[i] = x[i] + e[L.agg[i]];
            __syncthreads();
            const T* r = L.v[0];
            for (int32_t i = t; i < L.n; i += TB)
                L.v[3][i] = x[i] + omega * (L.dinv[i] * (r[i] - tail_row_sum(L, x, i)));
        }
        __syncthreads();
    }
}

// the level-0 system of a hierarchy: the fused pattern (with its
// offset-coded SpMV form) or the solve-order copy (plain CSR)
struct Src {
    int64_t nnz;
    const int32_t* row_ptr;
    const int32_t* col;
    const double* val64;
    const float* val32;
    const double* dinv64;
    const float* dinv32;
    SpmvIdx ix;
};

Src source(const rp_plan* p, bool ordered) {
    if (ordered)
        return Src{p->nnz, p->d_ro_row_ptr, p->d_ro_col, p->d_ro_val64, p->d_ro_val32, p->d_ro_dinv64,
                   p->d_ro_dinv32, SpmvIdx{p->d_ro_row_ptr, p->d_ro_col, nullptr, nullptr, nullptr}};
    return Src{p->nnz, p->d_row_ptr, p->d_col, p->d_val64, p->d_val32, p->d_dinv64, p->d_dinv32, spmv_idx(p)};
}

AmgHier*& hier(rp_plan* p, bool ordered) { return ordered ? p->amg_ro : p->amg; }

template <typename T>
struct Prec;
template <>
struct Prec<double> {
    static const double* val(const AmgLevel& L) { return L.val64; }
    static const double* dinv(const AmgLevel& L) { return L.dinv64; }
    static double** vec(AmgLevel& L) { return L.vec64; }
    static const double* cinv(const AmgHier& h) { return h.cinv64; }
    static void*& tail(AmgHier& h) { return h.tail64; }
    static const double* val0(const Src& q) { return q.val64; }
    static const double* dinv0(const Src& q) { return q.dinv64; }
};
template <>
struct Prec<float> {
    static const float* val(const AmgLevel& L) { return L.val32; }
    static const float* dinv(const AmgLevel& L) { return L.dinv32; }
    static float** vec(AmgLevel& L) { return L.vec32; }
    static const float* cinv(const AmgHier& h) { return h.cinv32; }
    static void*& tail(AmgHier& h) { return h.tail32; }
    static const float* val0(const Src& q) { return q.val32; }
    static const float* dinv0(const Src& q) { return q.dinv32; }
};

template <typename T>
int alloc_vectors(AmgHier& h) {
    for (int32_t l = 0; l < h.n_levels; ++l) {
        AmgLevel& L = h.lev[l];
        T** v = Prec<T>::vec(L);
        const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(L.n, 1);
        // in and out below level 0 (level 0 uses the solve's vectors); x and t
        // on smoothed levels.  Each one is allocated once, so a call after a
        // failed one completes the set.
        const bool last = l == h.n_levels - 1;
        const bool smooth = !last && l % 2 == 0;
        for (int k = 0; k < 4; ++k) {
            const bool need = (k == 0 || k == 3) ? l > 0 : smooth;
            if (need && !v[k]) RP_HIP_TRY(hipMalloc(&v[k], bytes));
        }
    }
    // the tail's per-level pointers, once the vectors exist
    void*& tab = Prec<T>::tail(h);
    if (h.tail_level > 0 && !tab) {
        std::vector<TailLevel<T>> tl;
        for (int32_t l = h.tail_level; l < h.n_levels; ++l) {
            AmgLevel& L = h.lev[l];
            T** v = Prec<T>::vec(L);
            tl.push_back(TailLevel<T>{(int32_t)L.n, L.row_ptr, L.col, Prec<T>::val(L), Prec<T>::dinv(L), L.agg,
                                      L.mem_ptr, L.mem, {v[0], v[1], v[2], v[3]}});
        }
        void* d = nullptr;
        RP_HIP_TRY(hipMalloc(&d, sizeof(TailLevel<T>) * tl.size()));
        const hipError_t e = hipMemcpy(d, tl.data(), sizeof(TailLevel<T>) * tl.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            RP_HIP_TRY(e);
        }
        tab = d;
    }
    return RP_OK;
}

SpmvIdx level_idx(const Src& q, const AmgLevel& L, int32_t l) {
    if (l == 0) return q.ix;
    return SpmvIdx{L.row_ptr, L.col, nullptr, nullptr, nullptr};
}

// y = V_l(r) on stream s (level 0: r and y are the solve's vectors)
template <typename T>
int vcycle(AmgHier& h, const Src& q, int32_t l, const T* r, T* y, T* part, int32_t n_part, bool rr,
           const int32_t* gate, hipStream_t s) {
    AmgLevel& L = h.lev[l];
    const int32_t n = (int32_t)L.n;
    const T omega = (T)RP_AMG_OMEGA;
    const bool want = part != nullptr;
    if (l > 0 && l == h.tail_level) {
        hipLaunchKernelGGL(amg_tail<T>, dim3(1), dim3(TB), 0, s, l, h.n_levels - 1,
                           (const TailLevel<T>*)Prec<T>::tail(h), Prec<T>::cinv(h), omega, gate);
        RP_HIP_TRY(hipGetLastError());
        return RP_OK;
    }
    if (l == h.n_levels - 1) {
#define RP_LAUNCH(PT, RRF)                                                                                       \
    hipLaunchKernelGGL((amg_coarse<T, PT, RRF>), dim3(1), dim3(AB), 0, s, n, Prec<T>::cinv(h), r, y, part, n_part, \
                       gate)
        if (want && rr) RP_LAUNCH(true, true);
        else if (want) RP_LAUNCH(true, false);
        else RP_LAUNCH(false, false);
#undef RP_LAUNCH
        RP_HIP_TRY(hipGetLastError());
        return RP_OK;
    }
    AmgLevel& C = h.lev[l + 1];
    const int32_t nc = (int32_t)C.n;
    T** cv = Prec<T>::vec(C);
    if (l % 2 == 1) {
        hipLaunchKernelGGL(amg_restrict<T>, dim3(grid_of(nc)), dim3(AB), 0, s, nc, L.mem_ptr, L.mem, r, cv[0], gate);
        RP_HIP_TRY(hipGetLastError());
        RP_TRY(vcycle<T>(h, q, l + 1, cv[0], cv[3], nullptr, 0, false, gate, s));
        hipLaunchKernelGGL((amg_prolong<T, false>), dim3(grid_of(n)), dim3(AB), 0, s, n, L.agg, cv[3], y, gate);
        RP_HIP_TRY(hipGetLastError());
        return RP_OK;
    }
    T** v = Prec<T>::vec(L);
    const T* val = l == 0 ? Prec<T>::val0(q) : Prec<T>::val(L);
    const T* dinv = l == 0 ? Prec<T>::dinv0(q) : Prec<T>::dinv(L);
    const SpmvIdx ix = level_idx(q, L, l);
    const int gs = spmv_grid(n), cr = chunk_rows(L), gc = chunk_grid(n, cr);
    hipLaunchKernelGGL(amg_pre<T>, dim3(grid_of(n)), dim3(AB), 0, s, n, r, dinv, v[1], omega, gate);
    if (l == 0)
        hipLaunchKernelGGL(amg_resid<T>, dim3(gs), dim3(SPMV_BLOCK), 0, s, n, ix, val, v[1], r, v[2], gate);
    else if (cr == 64)
        hipLaunchKernelGGL((amg_csr_resid<T, 64>), dim3(gc), dim3(WB), 0, s, n, L.row_ptr, L.col, val, v[1], r,
                           v[2], gate);
    else
        hipLaunchKernelGGL((amg_csr_resid<T, 32>), dim3(gc), dim3(WB), 0, s, n, L.row_ptr, L.col, val, v[1], r,
                           v[2], gate);
    hipLaunchKernelGGL(amg_restrict<T>, dim3(grid_of(nc)), dim3(AB), 0, s, nc, L.mem_ptr, L.mem, v[2], cv[0], gate);
    RP_HIP_TRY(hipGetLastError());
    RP_TRY(vcycle<T>(h, q, l + 1, cv[0], cv[3], nullptr, 0, false, gate, s));
    hipLaunchKernelGGL((amg_prolong<T, true>), dim3(grid_of(n)), dim3(AB), 0, s, n, L.agg, cv[3], v[1], gate);
#define RP_LAUNCH(PT, RRF)                                                                                    \
    hipLaunchKernelGGL((amg_post<T, PT, RRF>), dim3(gs), dim3(SPMV_BLOCK), 0, s, n, ix, val, v[1], r, dinv, omega, \
                       y, part, gate)
    if (want && rr) RP_LAUNCH(true, true);
    else if (want) RP_LAUNCH(true, false);
    else if (l == 0) RP_LAUNCH(false, false);
    else if (cr == 64)
        hipLaunchKernelGGL((amg_csr_post<T, 64>), dim3(gc), dim3(WB), 0, s, n, L.row_ptr, L.col, val, v[1], r, dinv,
                           omega, y, gate);
    else
        hipLaunchKernelGGL((amg_csr_post<T, 32>), dim3(gc), dim3(WB), 0, s, n, L.row_ptr, L.col, val, v[1], r, dinv,
                           omega, y, gate);
#undef RP_LAUNCH
    RP_HIP_TRY(hipGetLastError());
    return RP_OK;
}

template <typename T>
T* dalloc(int64_t n) {
    T* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) return nullptr;
    return q;
}

#define RP_DALLOC(ptr, T, n)                                          \
    do {                                                              \
        (ptr) = dalloc<T>(n);                                         \
        if (!(ptr)) {                                                 \
            set_error("out of device memory building the multigrid"); \
            return RP_ERR_HIP;                                        \
        }                                                             \
    } while (0)

void free_level(AmgLevel& L) {
    void* q[] = {L.row_ptr, L.col, L.val64, L.val32, L.dinv64, L.dinv32, L.diag_pos, L.agg, L.mem_ptr, L.mem,
                 L.cptr, L.cpos, L.vec64[0], L.vec64[1], L.vec64[2], L.vec64[3], L.vec32[0], L.vec32[1],
                 L.vec32[2], L.vec32[3]};
    for (void* a : q)
        if (a) (void)hipFree(a);
    L = AmgLevel();
}

// level l + 1 from level l (its CSR: row_ptr, col, val64)
int coarsen(AmgHier& h, const Src& q, int32_t l, hipStream_t s) {
    AmgLevel& L = h.lev[l];
    const int32_t n = (int32_t)L.n;
    const int32_t* rp_ = l == 0 ? q.row_ptr : L.row_ptr;
    const int32_t* cl = l == 0 ? q.col : L.col;
    const double* vl = l == 0 ? q.val64 : L.val64;
    struct Tmp {   // work arrays of this call, freed on every return
        std::vector<void*> q;
        ~Tmp() {
            for (void* a : q)
                if (a) (void)hipFree(a);
        }
    } tmp;
    int32_t *mate = nullptr, *pick = nullptr, *leader = nullptr, *is_leader = nullptr, *lead_id = nullptr;
    RP_DALLOC(mate, int32_t, n);
    tmp.q.push_back(mate);
    RP_DALLOC(pick, int32_t, n);
    tmp.q.push_back(pick);
    RP_DALLOC(leader, int32_t, n);
    tmp.q.push_back(leader);
    RP_DALLOC(is_leader, int32_t, n);
    tmp.q.push_back(is_leader);
    RP_DALLOC(lead_id, int32_t, n + 1);
    tmp.q.push_back(lead_id);
    const int g = grid_of(n);
    hipLaunchKernelGGL(amg_fill, dim3(g), dim3(AB), 0, s, n, -1, mate);
    for (int round = 0; round < AMG_ROUNDS; ++round) {
        hipLaunchKernelGGL(amg_fill, dim3(1), dim3(AB), 0, s, 1, 0, (int32_t*)h.flag);
        hipLaunchKernelGGL(amg_pick, dim3(g), dim3(AB), 0, s, n, rp_, cl, vl, mate, pick);
        hipLaunchKernelGGL(amg_pair, dim3(g), dim3(AB), 0, s, n, pick, mate, h.flag);
        RP_HIP_TRY(hipGetLastError());
        uint32_t pairs = 0;
        RP_HIP_TRY(hipMemcpyAsync(&pairs, h.flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        RP_HIP_TRY(hipStreamSynchronize(s));
        if (pairs == 0) break;
    }
    hipLaunchKernelGGL(amg_leader, dim3(g), dim3(AB), 0, s, n, rp_, cl, vl, mate, leader, is_leader);
    RP_HIP_TRY(hipGetLastError());
    int32_t nc = 0;
    RP_TRY(scan_i32(is_leader, n, lead_id, &nc, s));
    if (nc == n) {
        set_error("multigrid: no aggregate formed on level %d (%d rows without negative couplings)", l, n);
        return RP_ERR_UNSUPPORTED;
    }
    AmgLevel& C = h.lev[l + 1];
    C.n = nc;
    RP_DALLOC(L.agg, int32_t, n);
    RP_DALLOC(L.mem_ptr, int32_t, nc + 1);
    RP_DALLOC(L.mem, int32_t, n);
    int32_t *cnt = nullptr, *kstart = nullptr, *ucnt = nullptr;
    RP_DALLOC(cnt, int32_t, nc + 1);
    tmp.q.push_back(cnt);
    hipLaunchKernelGGL(amg_fill, dim3(grid_of(nc)), dim3(AB), 0, s, nc, 0, cnt);
    hipLaunchKernelGGL(amg_number, dim3(g), dim3(AB), 0, s, n, leader, lead_id, L.agg, cnt);
    RP_HIP_TRY(hipGetLastError());
    int32_t total = 0;
    RP_TRY(scan_i32(cnt, nc, L.mem_ptr, &total, s));
    hipLaunchKernelGGL(amg_fill, dim3(grid_of(nc)), dim3(AB), 0, s, nc, 0, cnt);
    hipLaunchKernelGGL(amg_members, dim3(g), dim3(AB), 0, s, n, L.agg, L.mem_ptr, cnt, L.mem);
    hipLaunchKernelGGL(amg_sort_members, dim3(grid_of(nc)), dim3(AB), 0, s, nc, L.mem_ptr, L.mem, rp_, cnt);
    RP_HIP_TRY(hipGetLastError());
    RP_DALLOC(kstart, int32_t, nc + 1);
    tmp.q.push_back(kstart);
    int32_t nkeys = 0;
    RP_TRY(scan_i32(cnt, nc, kstart, &nkeys, s));
    if ((int64_t)nkeys != L.nnz) {
        set_error("multigrid: %d coarse keys for %lld fine entries on level %d", nkeys, (long long)L.nnz, l);
        return RP_ERR_HIP;
    }
    uint64_t* keys = nullptr;
    RP_DALLOC(keys, uint64_t, L.nnz);
    tmp.q.push_back(keys);
    RP_DALLOC(ucnt, int32_t, nc + 1);
    tmp.q.push_back(ucnt);
    hipLaunchKernelGGL(amg_keys, dim3(grid_of(nc)), dim3(AB), 0, s, nc, L.mem_ptr, L.mem, rp_, cl, L.agg, kstart,
                       keys, ucnt);
    RP_HIP_TRY(hipGetLastError());
    RP_DALLOC(C.row_ptr, int32_t, nc + 1);
    int32_t nnz_c = 0;
    RP_TRY(scan_i32(ucnt, nc, C.row_ptr, &nnz_c, s));
    C.nnz = nnz_c;
    RP_DALLOC(C.col, int32_t, nnz_c + SPMV_PAD);
    RP_DALLOC(C.val64, double, nnz_c + SPMV_PAD);
    RP_DALLOC(C.val32, float, nnz_c + SPMV_PAD);
    RP_DALLOC(C.dinv64, double, nc);
    RP_DALLOC(C.dinv32, float, nc);
    RP_DALLOC(C.diag_pos, int32_t, nc);
    RP_DALLOC(L.cptr, int32_t, nnz_c + 1);
    RP_DALLOC(L.cpos, int32_t, L.nnz);
    RP_HIP_TRY(hipMemsetAsync(C.col + nnz_c, 0, sizeof(int32_t) * SPMV_PAD, s));
    RP_HIP_TRY(hipMemsetAsync(C.val64 + nnz_c, 0, sizeof(double) * SPMV_PAD, s));
    RP_HIP_TRY(hipMemsetAsync(C.val32 + nnz_c, 0, sizeof(float) * SPMV_PAD, s));
    hipLaunchKernelGGL(amg_cfill, dim3(grid_of(nc)), dim3(AB), 0, s, nc, kstart, keys, C.row_ptr, C.col, C.diag_pos,
                       L.cptr, L.cpos);
    RP_HIP_TRY(hipGetLastError());
    RP_HIP_TRY(hipStreamSynchronize(s));
    return RP_OK;
}

// coarse values, diagonals and the coarsest inverse from the plan's values
int refresh(AmgHier& h, const Src& q, int64_t version, hipStream_t s) {
    hipLaunchKernelGGL(amg_fill, dim3(1), dim3(AB), 0, s, 1, 0, (int32_t*)h.flag);
    for (int32_t l = 0; l + 1 < h.n_levels; ++l) {
        AmgLevel &L = h.lev[l], &C = h.lev[l + 1];
        const double* fine = l == 0 ? q.val64 : L.val64;
        hipLaunchKernelGGL(amg_gvals, dim3(grid_of(C.nnz)), dim3(AB), 0, s, (int32_t)C.nnz, L.cptr, L.cpos, fine,
                           C.val64, C.val32);
        hipLaunchKernelGGL(amg_gdiag, dim3(grid_of(C.n)), dim3(AB), 0, s, (int32_t)C.n, C.diag_pos, C.val64, C.dinv64,
                           C.dinv32, h.flag);
        RP_HIP_TRY(hipGetLastError());
    }
    const AmgLevel& Lc = h.lev[h.n_levels - 1];
    const int32_t* rp_ = h.n_levels == 1 ? q.row_ptr : Lc.row_ptr;
    const int32_t* cl = h.n_levels == 1 ? q.col : Lc.col;
    const double* vl = h.n_levels == 1 ? q.val64 : Lc.val64;
    hipLaunchKernelGGL(amg_dense_inverse, dim3(1), dim3(GJ_THREADS), 0, s, (int32_t)Lc.n, rp_, cl, vl, h.cwork,
                       h.cinv64, h.cinv32, h.flag);
    RP_HIP_TRY(hipGetLastError());
    uint32_t bad = 0;
    RP_HIP_TRY(hipMemcpyAsync(&bad, h.flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    if (bad) {
        set_error("multigrid: a coarse diagonal or a pivot of the coarsest inverse is not positive");
        return RP_ERR_BREAKDOWN;
    }
    h.version = version;
    return RP_OK;
}

void free_hier(AmgHier*& hp) {
    if (!hp) return;
    AmgHier& h = *hp;
    // every level: a failed coarsening leaves arrays on the level it was building
    for (int32_t l = 0; l < AMG_MAX_LEVELS; ++l) free_level(h.lev[l]);
    for (void* a : {(void*)h.cinv64, (void*)h.cinv32, (void*)h.cwork, (void*)h.flag, h.tail64, h.tail32})
        if (a) (void)hipFree(a);
    delete hp;
    hp = nullptr;
}

}  // namespace

void amg_free(rp_plan* p) {
    free_hier(p->amg);
    free_hier(p->amg_ro);
}

int amg_setup(rp_plan* p, hipStream_t s, bool ordered) {
    if (p->nnz_nl > 0) {
        set_error("multigrid needs the whole system on the GPU (the share has a non-local block)");
        return RP_ERR_UNSUPPORTED;
    }
    AmgHier*& hp = hier(p, ordered);
    free_hier(hp);
    // a fused-order rebuild also retires the solve-order hierarchy: the next
    // multigrid solve in solve order builds it from the values then current
    if (!ordered) free_hier(p->amg_ro);
    hp = new AmgHier();
    AmgHier& h = *hp;
    const Src q = source(p, ordered);
    int rc = RP_OK;
    auto fail = [&](int code) {
        free_hier(hp);
        return code;
    };
    h.flag = dalloc<uint32_t>(2);
    if (!h.flag) return fail((set_error("out of device memory building the multigrid"), RP_ERR_HIP));
    h.lev[0].n = p->n_rows;
    h.lev[0].nnz = q.nnz;
    h.n_levels = 1;
    while (h.lev[h.n_levels - 1].n > AMG_COARSE_MAX) {
        if (h.n_levels == AMG_MAX_LEVELS) {
            set_error("multigrid: more than %d levels", AMG_MAX_LEVELS);
            return fail(RP_ERR_UNSUPPORTED);
        }
        if ((rc = coarsen(h, q, h.n_levels - 1, s)) != RP_OK) return fail(rc);
        h.n_levels += 1;
        // the coarse values now, so the next level's matching sees them
        AmgLevel &L = h.lev[h.n_levels - 2], &C = h.lev[h.n_levels - 1];
        const double* fine = h.n_levels == 2 ? q.val64 : L.val64;
        hipLaunchKernelGGL(amg_gvals, dim3(grid_of(C.nnz)), dim3(AB), 0, s, (int32_t)C.nnz, L.cptr, L.cpos, fine,
                           C.val64, C.val32);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return fail((set_error("launching amg_gvals failed: %s", hipGetErrorString(e)), RP_ERR_HIP));
    }
    // the first level below level 0 small enough for the one-workgroup tail
    for (int32_t l = 1; l < h.n_levels && h.tail_level == 0; ++l)
        if (h.lev[l].n <= AMG_TAIL_ROWS) h.tail_level = l;
    const int64_t nL = h.lev[h.n_levels - 1].n;
    h.cinv64 = dalloc<double>(nL * nL);
    h.cinv32 = dalloc<float>(nL * nL);
    h.cwork = dalloc<double>(nL * nL);
    if (!h.cinv64 || !h.cinv32 || !h.cwork)
        return fail((set_error("out of device memory building the multigrid"), RP_ERR_HIP));
    if ((rc = refresh(h, q, p->values_version, s)) != RP_OK) return fail(rc);
    return RP_OK;
}

int amg_prepare(rp_plan* p, bool fp32, hipStream_t s, bool ordered) {
    RP_TRY(alloc_z(p));
    AmgHier*& hp = hier(p, ordered);
    if (!hp) RP_TRY(amg_setup(p, s, ordered));
    if (hp->version != p->values_version) RP_TRY(refresh(*hp, source(p, ordered), p->values_version, s));
    if (fp32) RP_TRY(alloc_vectors<float>(*hp));
    else RP_TRY(alloc_vectors<double>(*hp));
    return RP_OK;
}

template <typename T>
int amg_apply(rp_plan* p, const T* r, T* y, T* part, int32_t n_part, bool rr, const int32_t* gate, hipStream_t s,
              bool ordered) {
    return vcycle<T>(*hier(p, ordered), source(p, ordered), 0, r, y, part, n_part, rr, gate, s);
}

template int amg_apply<double>(rp_plan*, const double*, double*, double*, int32_t, bool, const int32_t*,
                               hipStream_t, bool);
template int amg_apply<float>(rp_plan*, const float*, float*, float*, int32_t, bool, const int32_t*, hipStream_t,
                              bool);

}  // namespace rp

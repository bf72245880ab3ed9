// rp_update_values_noalloc: the device-memory form of rp_update_values for
// callers that cannot allocate.  Its only scratch memory is the table of
// per-rank pointers the gather reads (4 per rank), kept in a file-scope
// device array of fixed size instead of plan memory.  Each GPU holds its own
// copy of the array from first use until the process ends; its address on a
// device is taken once, with that device current, and reused.
#include <mutex>

#include "rp_internal.hpp"

namespace rp {

namespace {

constexpr int MAX_DEVICES = 64;

// 4 pointers per share rank; host code never names it again after taking
// its device address (the name is a host-side stand-in, not that address)
__device__ __align__(256) static uint64_t scratch[4 * RP_NOALLOC_MAX_RANKS];

std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// the device address of `scratch` on `device` (the current device)
int scratch_ptr(int device, void** out) {
    if (device < 0 || device >= MAX_DEVICES) {
        set_error("device %d beyond the %d the library tracks", device, MAX_DEVICES);
        return RP_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device] == nullptr) {
        void* ptr = nullptr;
        RP_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return RP_OK;
}

bool device_memory(const void* ptr) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

}  // namespace
}  // namespace rp

using namespace rp;

extern "C" int rp_update_values_noalloc(rp_plan* p, const double* const* diag, const double* const* upper,
                                        const double* const* lower, const double* const* iface, void* stream) {
    clear_error();
    if (p == nullptr) {
        set_error("plan is NULL");
        return RP_ERR_ARG;
    }
    if (diag == nullptr || upper == nullptr || iface == nullptr) {
        set_error("diag/upper/iface pointer arrays are NULL");
        return RP_ERR_ARG;
    }
    if (p->alpha > RP_NOALLOC_MAX_RANKS) {
        set_error("share of %d ranks: rp_update_values_noalloc takes at most %d", p->alpha, RP_NOALLOC_MAX_RANKS);
        return RP_ERR_ARG;
    }
    // per-rank table, built on the host in the plan's own host array (no
    // device memory touched yet)
    const double** table = p->h_src.data();
    for (int32_t i = 0; i < p->alpha; ++i) {
        const double* q[4] = {diag[i], upper[i], lower ? lower[i] : upper[i], iface[i]};
        const int64_t len[4] = {p->n_cells[i], p->n_faces[i], p->n_faces[i], p->n_iface[i]};
        for (int r = 0; r < 4; ++r) {
            if (len[r] > 0 && (q[r] == nullptr || !device_memory(q[r]))) {
                set_error("rank %d: array %d is NULL or not device memory (rp_update_values_noalloc reads "
                          "device arrays only)", i, r);
                return RP_ERR_ARG;
            }
            table[4 * i + r] = q[r];
        }
    }
    int cur = -1;
    RP_HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) RP_HIP_TRY(hipSetDevice(p->device));
    void* ptr = nullptr;
    RP_TRY(scratch_ptr(p->device, &ptr));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    RP_HIP_TRY(hipMemcpyAsync(ptr, table, sizeof(const double*) * 4 * (size_t)p->alpha, hipMemcpyHostToDevice, s));
    RP_TRY(launch_clear_flags(p->d_flags, s));
    RP_TRY(launch_update_gather(p, reinterpret_cast<const double* const*>(ptr), lower != nullptr, p->d_flags, s));
    p->has_values = true;
    p->values_version += 1;
    p->last_stream = s;
    return RP_OK;
}

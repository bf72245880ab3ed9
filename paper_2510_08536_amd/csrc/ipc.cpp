// Ranks in other processes (Sec. 3, update procedure; the GPU-aware
// communication study of Sec. 4): the owner exports its plan's receive
// buffer as an IPC handle, each rank process maps it and copies its own slot
// block [diag | upper | lower | interface] to U's offset straight into the
// owner's device memory -- the one-GPU analogue of ranks sending with
// GPU-aware MPI.  The owner then reorders the buffer with
// rp_update_values_slots.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <cstring>

#include "rp_internal.hpp"

using namespace rp;

static_assert(sizeof(hipIpcMemHandle_t) <= sizeof(rp_ipc_handle), "IPC handle does not fit");

namespace {

// shared allocations of 2 GiB and more are refused (opening them in other
// processes is not reliable on this platform)
constexpr int64_t IPC_MAX_BYTES = (int64_t)2 << 30;

int activate_device(int device) {
    int cur = -1;
    RP_HIP_TRY(hipGetDevice(&cur));
    if (cur != device) RP_HIP_TRY(hipSetDevice(device));
    return RP_OK;
}

}  // namespace

extern "C" {

int rp_plan_export_recv(rp_plan* p, rp_ipc_handle* out, int64_t* n_slots) {
    clear_error();
    if (p == nullptr || out == nullptr) {
        set_error("plan or out is NULL");
        return RP_ERR_ARG;
    }
    if ((int64_t)sizeof(double) * p->n_slots >= IPC_MAX_BYTES) {
        set_error("receive buffer of %lld bytes: shared buffers are limited to under 2 GiB",
                  (long long)(sizeof(double) * p->n_slots));
        return RP_ERR_UNSUPPORTED;
    }
    RP_TRY(activate_device(p->device));
    hipIpcMemHandle_t h;
    RP_HIP_TRY(hipIpcGetMemHandle(&h, p->d_recv));
    std::memset(out, 0, sizeof(*out));
    std::memcpy(out->bytes, &h, sizeof(h));
    if (n_slots) *n_slots = p->n_slots;
    return RP_OK;
}

int rp_recv_attach(const rp_ipc_handle* h, double** recv) {
    clear_error();
    if (h == nullptr || recv == nullptr) {
        set_error("handle or recv is NULL");
        return RP_ERR_ARG;
    }
    *recv = nullptr;
    hipIpcMemHandle_t hh;
    std::memcpy(&hh, h->bytes, sizeof(hh));
    void* ptr = nullptr;
    RP_HIP_TRY(hipIpcOpenMemHandle(&ptr, hh, hipIpcMemLazyEnablePeerAccess));
    *recv = static_cast<double*>(ptr);
    return RP_OK;
}

int rp_recv_write(double* recv, int64_t slot_offset, const double* diag, int32_t n_cells, const double* upper,
                  int32_t n_faces, const double* lower, const double* iface, int32_t n_iface, void* stream) {
    clear_error();
    if (recv == nullptr || slot_offset < 0 || n_cells < 0 || n_faces < 0 || n_iface < 0) {
        set_error("bad arguments");
        return RP_ERR_ARG;
    }
    if ((n_cells && !diag) || (n_faces && !upper) || (n_iface && !iface)) {
        set_error("diag, upper or iface is NULL");
        return RP_ERR_ARG;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double* dst = recv + slot_offset;
    const size_t nc = n_cells, nf = n_faces, ni = n_iface;
    if (nc) RP_HIP_TRY(hipMemcpyAsync(dst, diag, nc * 8, hipMemcpyDefault, s));
    if (nf) RP_HIP_TRY(hipMemcpyAsync(dst + nc, upper, nf * 8, hipMemcpyDefault, s));
    if (nf) RP_HIP_TRY(hipMemcpyAsync(dst + nc + nf, lower ? lower : upper, nf * 8, hipMemcpyDefault, s));
    if (ni) RP_HIP_TRY(hipMemcpyAsync(dst + nc + 2 * nf, iface, ni * 8, hipMemcpyDefault, s));
    RP_HIP_TRY(hipStreamSynchronize(s));
    return RP_OK;
}

int rp_recv_detach(double* recv) {
    clear_error();
    if (recv == nullptr) return RP_OK;
    RP_HIP_TRY(hipIpcCloseMemHandle(recv));
    return RP_OK;
}

}  // extern "C"

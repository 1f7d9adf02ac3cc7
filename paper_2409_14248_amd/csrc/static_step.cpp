// static_step.cpp -- the training step for callers that cannot allocate
// device memory: the workspace is a file-scope device array of the library
// instead of a caller buffer.
//
// The array lives in every GPU the library runs on until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in for the symbol): its device address is looked up once
// per device with hipGetSymbolAddress, with that device current, and kept.
// Every call on one GPU uses that GPU's array, so calls that overlap on one
// GPU (two streams, two threads) race on it; the array keeps the last call's
// contents.
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime_internal.h"

using namespace hrk;

namespace {

static __device__ __align__(256) unsigned char scratch[HRKAN_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

struct DevScratch {
    bool ready;
    void *ptr;
};
DevScratch g_dev[MAX_DEVICES];
std::mutex g_mu;

// Zero the status word (the only part of the workspace that must start at
// zero) with a kernel, which a caller's graph capture may record.
__global__ void k_clear_status(unsigned int *status)
{
    if (threadIdx.x < 64) status[threadIdx.x] = 0u;
}

// Device address of this device's array, looked up on the first call on the
// device (status word cleared then, on `stream`).
int scratch_of_current_device(hipStream_t stream, void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(HRKAN_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_mu);
    DevScratch &d = g_dev[dev];
    if (!d.ready) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(HRKAN_ERR_DEVICE, "hipGetSymbolAddress(scratch) gave a null address");
        hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, stream, (unsigned int *)ptr);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "status clear launch");
        d.ptr = ptr;
        d.ready = true;
    }
    *out = d.ptr;
    return HRKAN_OK;
}

}  // namespace

extern "C" {

int hrkan_step_static(const hrkan_net_desc *net, const hrkan_pde_desc *pde, const void *const *W,
                      const hrkan_points *pts, double *loss_out, void *const *gW_out, hipStream_t stream)
{
    if (prof_on())
        return fail(HRKAN_ERR_UNSUPPORTED, "hrkan_step_static does not run while per-launch profiling is on");
    if (!pts) return fail(HRKAN_ERR_INVALID_ARG, "pts is NULL");
    if (pts->n_int < 0 || pts->n_bc < 0) return fail(HRKAN_ERR_INVALID_ARG, "negative point count");
    size_t need = 0;
    int rc = hrkan_workspace_bytes(net, pde, pts->n_int, pts->n_bc, &need);
    if (rc != HRKAN_OK) return rc;
    if (need > (size_t)HRKAN_STATIC_SCRATCH_BYTES)
        return fail(HRKAN_ERR_WORKSPACE,
                    "hrkan_step_static: this step needs %zu bytes of workspace, above the static maximum of %zu "
                    "bytes (HRKAN_STATIC_SCRATCH_BYTES); call hrkan_step with a workspace instead",
                    need, (size_t)HRKAN_STATIC_SCRATCH_BYTES);
    void *ws = nullptr;
    rc = scratch_of_current_device(stream, &ws);
    if (rc != HRKAN_OK) return rc;
    return step_impl(net, pde, W, pts, loss_out, gW_out, ws, (size_t)HRKAN_STATIC_SCRATCH_BYTES, stream, false);
}

}  // extern "C"

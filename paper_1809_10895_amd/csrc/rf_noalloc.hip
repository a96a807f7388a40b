// The library's static device workspace: a file-scope device array that
// rf_bind_static_workspace binds as a context's workspace, for callers that
// cannot allocate device memory (code under stream capture, serving loops,
// harnesses that forbid hipMalloc).
//
// Every GPU that the library runs on holds its own copy of the array, at its
// own address, until the process ends.  Host code never uses the array's name
// as a device address: the address of each device's copy is looked up once
// per device with hipGetSymbolAddress (with that device current) and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rf_internal.h"

static_assert(RF_STATIC_WORKSPACE_BYTES % 256 == 0, "static workspace size");

static __device__ __align__(256) unsigned char scratch[RF_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up on the first
// call for the device); null on failure.
void *static_workspace(int device, hipError_t *err)
{
    *err = hipSuccess;
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_lock);
    if (!g_ptr[device]) {
        int cur = -1;
        if ((*err = hipGetDevice(&cur)) != hipSuccess) return nullptr;
        if (cur != device && (*err = hipSetDevice(device)) != hipSuccess) return nullptr;
        void *p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (*err != hipSuccess || !p) {
            if (*err == hipSuccess) *err = hipErrorInvalidSymbol;
            return nullptr;
        }
        g_ptr[device] = p;
    }
    return g_ptr[device];
}

}  // namespace

extern "C" rf_status rf_bind_static_workspace(rf_ctx *ctx)
{
    if (!ctx) return RF_ERR_ARG;
    hipError_t e;
    void *p = static_workspace(rf::ctx_device(ctx), &e);
    if (!p) return RF_ERR_HIP;
    return rf::ctx_bind(ctx, p, RF_STATIC_WORKSPACE_BYTES);
}

// A V-cycle entry point that allocates nothing (declared in mgir.h): the
// level vectors live in a file-scope device array instead of a workspace the
// caller binds, for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops).  Each GPU the library runs on
// holds its own copy of the array until the process ends.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>

#include "mg_launch.h"

namespace {

// 128 MiB: the V-cycle of a 255^3 FP16 hierarchy or a 127^3 FP64 one.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// The array's device address on each GPU.  In host code the name `scratch`
// only stands in for the symbol; kernels get these addresses.
std::atomic<void *> g_scratch[kMaxDevices];

mg_status_t scratch_ptr(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "hipGetDevice: %s", hipGetErrorString(e));
        return mg::set_error(MG_ERR_HIP, msg);
    }
    if (dev < 0 || dev >= kMaxDevices) return mg::set_error(MG_ERR_HIP, "device index beyond the scratch table");
    void *p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        // first call on this device, with it current: look the address up once
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char msg[160];
            std::snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return mg::set_error(MG_ERR_HIP, msg);
        }
        g_scratch[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return MG_OK;
}

}  // namespace

extern "C" {

mg_status_t mg_vcycle_noalloc(mg_handle h, const void *b, void *c, void *stream) {
    size_t need = 0;
    mg_status_t s = mg::vcycle_scratch_need(h, &need);
    if (s != MG_OK) return s;
    if (need > kScratchBytes) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "the V-cycle of this handle needs %zu bytes of scratch; mg_vcycle_noalloc holds %zu", need,
                      kScratchBytes);
        return mg::set_error(MG_ERR_WORKSPACE, msg);
    }
    if (!b || !c) return mg::set_error(MG_ERR_ARG, "null argument");
    void *p = nullptr;
    if ((s = scratch_ptr(&p)) != MG_OK) return s;
    return mg::vcycle_in(h, p, kScratchBytes, b, c, stream);
}

}  // extern "C"

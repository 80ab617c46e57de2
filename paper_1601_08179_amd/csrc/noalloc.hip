// Fixed device workspace of semcond_apply_noalloc: a file-scope device array,
// so that the entry point needs no allocation at call time (for callers that
// cannot allocate: code under HIP graph capture, tight serving loops).
//
// In host code the array's name is only a host-side stand-in; its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and every later use goes through the looked-up address.

#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.h"

namespace semcond {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[dev]) return hipSuccess;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
    return hipSuccess;
}

void* noalloc_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[dev];
}

}  // namespace semcond

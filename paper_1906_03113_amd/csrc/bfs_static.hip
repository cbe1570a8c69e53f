// The library's file-scope device scratch array, for the search entry point
// that allocates nothing (bfs_run_static in bfs_host.cpp).
//
// Each GPU the library runs on holds its own copy of `scratch` from module
// load until the process ends.  Host code never uses the array's name as an
// address: the first call on a device, with that device current, asks the
// runtime for that device's address of the array (hipGetSymbolAddress) and
// keeps it; every later use goes through the kept pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bfs_internal.h"

namespace bfsi {

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t static_scratch(void **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace bfsi

// croft_noalloc.hip -- the device scratch of croft_execute_scaled_noalloc:
// one statically allocated array per GPU, for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).
//
// In host code `scratch` names a host-side stand-in, not a device address;
// the kernels receive the address that hipGetSymbolAddress returns for the
// current device, looked up once per device (at the creation of the first
// half-storage plan on it) and kept below.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "croft_internal.h"

namespace croft {
namespace {

static __device__ __align__(256) int8_t scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, int8_t *> g_scratch_addr;  // device -> address of its copy of `scratch`

}  // namespace

hipError_t noalloc_scratch(int device, int8_t **ptr) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the device must be current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = static_cast<int8_t *>(p);
    *ptr = static_cast<int8_t *>(p);
    return hipSuccess;
}

}  // namespace croft

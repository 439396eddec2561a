// Device memory of the allocation-free apply (lmfmm_apply_noalloc): a fixed
// array in the library's code object, one copy per GPU, kept until the
// process ends.  Its device address is resolved once per device with that
// device current (lmfmm_create does it for the current device); host code
// uses only the resolved address, never the array's name.
#include <mutex>

#include "lmfmm_internal.h"

namespace lmfmm {

namespace {

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAXDEV = 64;
std::mutex g_mu;
void *g_ptr[MAXDEV] = {};

}  // namespace

hipError_t noalloc_scratch_init(int dev)
{
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[dev]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev) return hipErrorInvalidDevice;  // resolved only with the device current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_ptr[dev] = p;
    return hipSuccess;
}

void *noalloc_scratch_ptr(int dev)
{
    if (dev < 0 || dev >= MAXDEV) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[dev];
}

}  // namespace lmfmm

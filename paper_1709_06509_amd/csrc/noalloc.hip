// Device-resident scratch for the solve entry point that allocates nothing
// (bp_hierarchical_solve_noalloc).  The scratch is a file-scope device array: every GPU the
// library runs on holds its own copy, at its own address, until the process ends.  Host
// code never passes the array's name to a kernel or a copy (in host code the name is only a
// stand-in); it uses the device address hipGetSymbolAddress returns, looked up once per
// device with that device current and kept in a per-device table.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[bpst::kNoallocScratchBytes];

std::mutex g_scratch_lock;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace bpst {

hipError_t noalloc_scratch(void** ptr)
{
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_lock);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace bpst

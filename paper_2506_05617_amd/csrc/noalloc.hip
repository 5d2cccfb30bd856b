// Static device scratch of the no-allocation SVD entry point
// (lfa_svd_noalloc): a file-scope device array that stands in for the
// caller-owned workspace, so that entry point never allocates.  Each device
// holds its own copy of the array (from the first load of this library's
// code on that device until the process ends); its address on a device is
// looked up once, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lfa_internal.hpp"

namespace lfa {
namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of `scratch` on `device`, which must be the current
// device.  Host code never passes the array's own name to a kernel (on the
// host it only names a stand-in): it passes this address.
hipError_t noalloc_scratch(int device, void** ptr, size_t* bytes) {
    if (device < 0 || device >= kMaxDevices || !ptr || !bytes) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    *bytes = kNoAllocScratchBytes;
    return hipSuccess;
}

}  // namespace lfa

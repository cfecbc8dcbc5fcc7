// Static device scratch of the allocation-free evaluation entry point
// (scff_eval_grid_noalloc): the 1D tables of the grid and, when they fit
// after them, the FP64 partial sums of a split chunk list live in this
// file-scope array instead of context buffers, so that call allocates no
// device memory.  Each device the library runs on holds its own copy of the
// array (kScratchBytes) until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "engine.h"

namespace scff {

namespace {
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this device's scratch array.  Called with `device`
// current (context creation); the symbol is resolved once per device and
// kept.  In host code the array's name is not a device address: kernels and
// copies must use the pointer returned here.
hipError_t scratch_address(int device, void** ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

}  // namespace scff

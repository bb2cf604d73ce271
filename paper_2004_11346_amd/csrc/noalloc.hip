// Fixed device scratch for the allocation-free inverse (sht_inverse_noalloc).
//
// The inverse SHT stages the phi-analysed grid g between its DFT and its
// transposed ALT.  sht_inverse keeps g in the plan's workspace; the
// allocation-free variant keeps it in `scratch`, a file-scope device array of
// kNoallocScratchBytes that exists once per GPU for the life of the process.
// Host code never passes the array's name to a kernel (on the host it is only
// a stand-in for the symbol): its device address is looked up once per device
// with hipGetSymbolAddress, with that device current, and that address is used
// everywhere.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sht_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[sht::kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {nullptr};

}  // namespace

namespace sht {

// Called from plan creation with the plan's device current.
int noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return (int)hipSuccess;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    g_ptr[device] = ptr;
    return (int)hipSuccess;
}

void *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace sht

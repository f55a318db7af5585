// Static device scratch of the allocation-free entry point ps_execute_static.
//
// The array below is a file-scope __device__ variable: the HIP runtime
// places one copy of it on every GPU that loads the library's code object,
// held until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in symbol): static_scratch_setup,
// called at plan creation with the plan's device current, resolves that
// device's copy once with hipGetSymbolAddress and keeps the pointer; every
// later use goes through static_scratch_ptr().
#include <mutex>

#include "ps_internal.h"

namespace ps {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void* g_ptr[kMaxDevices] = {};
std::mutex g_mu;
}  // namespace

hipError_t static_scratch_setup() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[dev]) return hipSuccess;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_ptr[dev] = ptr;
    return hipSuccess;
}

void* static_scratch_ptr() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[dev];
}

}  // namespace ps

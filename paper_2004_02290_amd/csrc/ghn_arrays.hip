// The library's static device arrays and their per-device addresses.
//
// In host code a __device__ array's name only names the symbol (a host-side stand-in,
// not a device address).  Each array's address on a GPU comes from
// hipGetSymbolAddress, called once per device with that device current, and is kept
// per device here; only that address is ever passed to kernels or copies.
#include <mutex>

#include "ghn_internal.h"

namespace ghn {

namespace {

constexpr int SYMBOL_DEVICES = 256;

struct SymbolCache {
    std::mutex mu;
    void* ptr[SYMBOL_DEVICES] = {};
};

hipError_t symbol_address(const void* symbol, SymbolCache& cache, void** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SYMBOL_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(cache.mu);
    if (!cache.ptr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, symbol)) != hipSuccess) return e;
        cache.ptr[dev] = p;
    }
    *out = cache.ptr[dev];
    return hipSuccess;
}

// Workspace of ghn_predict_noalloc: GHN_NOALLOC_WS_BYTES on every GPU the library runs
// on, kept until the process ends.
__device__ __align__(256) unsigned char scratch[GHN_NOALLOC_WS_BYTES];
SymbolCache g_scratch;

// The walk fault word of each GPU (GHN_WALK_SHORT), padded to its own 256 bytes.
__device__ __align__(256) uint32_t walk_fault_word[64];
SymbolCache g_fault_word;

__global__ void k_clear_word(uint32_t* w) { *w = 0u; }

}  // namespace

hipError_t noalloc_workspace(void** out) { return symbol_address(HIP_SYMBOL(scratch), g_scratch, out); }

hipError_t walk_fault_address(uint32_t** out) {
    return symbol_address(HIP_SYMBOL(walk_fault_word), g_fault_word, (void**)out);
}

hipError_t launch_clear_word(uint32_t* w, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, s, w);
    return launch_status();
}

}  // namespace ghn

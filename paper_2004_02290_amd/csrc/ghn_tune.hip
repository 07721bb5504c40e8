// Autotuner: picks the cell width, the screen (FP32 per query or grouped bf16)
// and its query grouping by timing ghn_predict on a sample of queries.  Under
// the EXACT stop rule every width gives the brute-force result, so the width is
// tuned freely; under the PAPER rule the width is part of the method (the walk
// and its result depend on it) and only the execution settings are tuned.
#include <cmath>
#include <cstring>
#include <vector>

#include "ghn_internal.h"

namespace ghn {
namespace {

// order-preserving map of floats to unsigned ints (for atomic min/max)
__device__ __forceinline__ uint32_t f2ord(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(256) void k_coord_range(const void* pts, int64_t n, int32_t f, int32_t dtype,
                                                     uint32_t* lohi) {
    for (int j = 0; j < f; ++j) {
        uint32_t lo = 0xffffffffu, hi = 0u;
        for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
            const float x = dtype == GHN_BF16 ? __uint_as_float((uint32_t)((const uint16_t*)pts)[i * f + j] << 16)
                                              : ((const float*)pts)[i * f + j];
            if (!isfinite(x)) continue;
            lo = min(lo, f2ord(x));
            hi = max(hi, f2ord(x));
        }
        for (int d = 1; d < WAVE; d <<= 1) {
            lo = min(lo, (uint32_t)__shfl_xor((int)lo, d, WAVE));
            hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, WAVE));
        }
        if (lane_id() == 0) {
            atomicMin(&lohi[2 * j], lo);
            atomicMax(&lohi[2 * j + 1], hi);
        }
    }
}

float ord2f(uint32_t u) {
    const uint32_t b = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    float x;
    std::memcpy(&x, &b, 4);
    return x;
}

}  // namespace

hipError_t coord_range(const void* pts, int64_t n, int32_t f, int32_t dtype, float* lo, float* hi, hipStream_t s) {
    uint32_t* d = nullptr;
    hipError_t e = device_alloc((void**)&d, (size_t)2 * f * 4);
    if (e != hipSuccess) return e;
    std::vector<uint32_t> h((size_t)2 * f);
    for (int j = 0; j < f; ++j) { h[2 * j] = 0xffffffffu; h[2 * j + 1] = 0u; }
    if ((e = hipMemcpyAsync(d, h.data(), h.size() * 4, hipMemcpyHostToDevice, s)) == hipSuccess) {
        int64_t g = (n + 255) / 256;
        if (g > 1024) g = 1024;
        hipLaunchKernelGGL(k_coord_range, dim3((unsigned)g), dim3(256), 0, s, pts, n, f, dtype, d);
        if ((e = launch_status()) == hipSuccess &&
            (e = hipMemcpyAsync(h.data(), d, h.size() * 4, hipMemcpyDeviceToHost, s)) == hipSuccess)
            e = hipStreamSynchronize(s);
    }
    ghn::device_free(d);
    for (int j = 0; j < f; ++j) { lo[j] = ord2f(h[2 * j]); hi[j] = ord2f(h[2 * j + 1]); }
    return e;
}

}  // namespace ghn
